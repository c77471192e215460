"""Oracle: Jacobian-vector products and the sparse Jacobian of F.

TEST INFRASTRUCTURE ONLY.

* ``jvp_fd``: finite-difference product (Sect. 4.2, eq. jacobian_free) with the perturbation
  of eq. pert_old, delta = lam (lam + ||x||/||v||).  The norms are 2-norms of the vectors in
  the scaled space of eq. jacobian_system_norm (x = R^-1 X, v = R^-1 dX), so delta is
  unit-free.  lam = 1e-7 is the value the Results section finds necessary at low Mach.
* ``jvp_cs``: exact product by the complex step Im F(X + i h v)/h, h = 1e-200 (frozen
  branches; see H_CS).
* ``jacobian_sparse``: the full sparse Jacobian, columns from complex steps on coloured
  groups of unknowns.  The stencil reaches cells at offsets -3..+3 per axis, so cells whose
  indices agree modulo a period P >= 8 (P divides n on periodic axes) never share a row.
  Axes where no such P exists use one colour per cell (brute force).

Pins (tests/test_oracle_jacobian.py): the complex step equals a brute-force central
difference dense Jacobian on tiny grids; J.v from the sparse Jacobian equals jvp_cs; the
finite-difference product converges to it at the rate O(delta).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .residual import Problem, residual_F, WALL
from .scaling import scaling_LR

# Complex-step size.  Products of two imaginary parts (h^2 ~ 1e-400) underflow to exactly
# zero, so the real part of every intermediate equals the real evaluation and every upwind /
# limiter branch is taken exactly as in the real computation (frozen branches).  With a
# larger h (e.g. 1e-30) the O(h^2) real corrections decide exact ties such as a zero mass
# flux on a plane where u = 0, making the "derivative" depend on the direction.
H_CS = 1e-200


def fd_delta(prob: Problem, X, v, lam=1e-7, alpha1=1e-5, alpha2=1.0):
    """Perturbation size of eq. pert_old with scaled 2-norms."""
    _, R = scaling_LR(prob, X, alpha1, alpha2)
    nx = np.linalg.norm((X / R).ravel())
    nv = np.linalg.norm((v / R).ravel())
    if nv == 0.0:
        return 0.0
    return lam * (lam + nx / nv)


def jvp_fd(prob: Problem, X, b, dt, v, lam=1e-7, F0=None, alpha1=1e-5, alpha2=1.0):
    """(F(X + delta v) - F(X)) / delta (eq. jacobian_free)."""
    delta = fd_delta(prob, X, v, lam, alpha1, alpha2)
    if delta == 0.0:
        return np.zeros_like(X)
    if F0 is None:
        F0 = residual_F(prob, X, b, dt)
    return (residual_F(prob, X + delta * v, b, dt) - F0) / delta


def jvp_cs(prob: Problem, X, b, dt, v):
    """Exact J v = Im F(X + i h v)/h."""
    Fc = residual_F(prob, X.astype(np.complex128) + 1j * H_CS * v, b, dt)
    return np.imag(Fc) / H_CS


def colour_period(n, bc, min_period=8):
    if bc == WALL:
        return min(n, min_period)
    for P in range(min_period, n + 1):
        if n % P == 0:
            return P
    return n


def jacobian_sparse(prob: Problem, X, b, dt):
    """Sparse J = dF/dX (CSR, rows and columns in the flattened layout of X)."""
    nd = prob.nd
    nv = prob.nvar
    fs = prob.field_shape
    N = prob.ncell
    n_unk = nv * N
    periods = [colour_period(prob.shape[d], prob.bc[d]) for d in range(nd)]
    # per-axis coordinate grids of every cell (field orientation)
    grids = np.meshgrid(*[np.arange(n) for n in fs], indexing="ij")
    coord = [grids[prob.axis(d)] for d in range(nd)]  # coord[d] = index along axis d
    rows_all, cols_all, vals_all = [], [], []
    Xc = X.astype(np.complex128)
    import itertools
    for col_var in range(nv):
        for residues in itertools.product(*[range(P) for P in periods]):
            mask = np.ones(fs, dtype=bool)
            for d in range(nd):
                mask &= (coord[d] % periods[d]) == residues[d]
            pert = np.zeros(X.shape)
            pert[col_var][mask] = 1.0
            Fi = np.imag(residual_F(prob, Xc + 1j * H_CS * pert, b, dt)) / H_CS
            nz = np.nonzero(Fi)
            if len(nz[0]) == 0:
                continue
            vals = Fi[nz]
            row_var = nz[0]
            row_cell = nz[1:]
            # locate the coloured column that reaches this row: per axis, the unique index
            # congruent to the residue within distance 3 of the row's cell
            col_idx = []
            for d in range(nd):
                a = prob.axis(d)
                n = prob.shape[d]
                P = periods[d]
                rc = row_cell[a]
                if P == n:
                    ci = np.full_like(rc, residues[d])
                else:
                    base = rc - 3
                    ci = base + np.mod(residues[d] - base, P)
                    if prob.bc[d] != WALL:
                        ci = np.mod(ci, n)
                col_idx.append(ci)
            cell_lin = np.ravel_multi_index(tuple(col_idx[d] for d in reversed(range(nd))), fs)
            row_lin = np.ravel_multi_index(row_cell, fs)
            rows_all.append(row_var * N + row_lin)
            cols_all.append(col_var * N + cell_lin)
            vals_all.append(vals)
    rows = np.concatenate(rows_all)
    cols = np.concatenate(cols_all)
    vals = np.concatenate(vals_all)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n_unk, n_unk))


def jacobian_dense_cs(prob: Problem, X, b, dt):
    """Dense J, one complex step per unknown (tiny grids only)."""
    n_unk = X.size
    J = np.empty((n_unk, n_unk))
    Xc = X.astype(np.complex128)
    for k in range(n_unk):
        pert = np.zeros(n_unk)
        pert[k] = 1.0
        Fi = residual_F(prob, Xc + 1j * H_CS * pert.reshape(X.shape), b, dt)
        J[:, k] = (np.imag(Fi) / H_CS).ravel()
    return J


def jacobian_dense_central(prob: Problem, X, b, dt, eps=1e-6):
    """Dense J by central real differences, step eps*max(1,|x_k|) (tiny grids only)."""
    n_unk = X.size
    J = np.empty((n_unk, n_unk))
    x = X.ravel()
    for k in range(n_unk):
        h = eps * max(1.0, abs(x[k]))
        xp = x.copy()
        xm = x.copy()
        xp[k] += h
        xm[k] -= h
        Fp = residual_F(prob, xp.reshape(X.shape), b, dt)
        Fm = residual_F(prob, xm.reshape(X.shape), b, dt)
        J[:, k] = ((Fp - Fm) / (2 * h)).ravel()
    return J
