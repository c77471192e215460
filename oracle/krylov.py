"""Oracle: right-preconditioned flexible GMRES(m) with classical Gram-Schmidt applied twice.

TEST INFRASTRUCTURE ONLY.

GMRES with zero initial guess, stopped when ||A x - b||_2 < eta ||b||_2 (Sect. 4.1,
eq. forcing_term), right preconditioning (Sect. 4.3, eqs. lin_sys_rp, lin_sys_rp2).  Readings
where the paper is silent: the preconditioned directions z_j = M^-1 v_j are stored (flexible
GMRES, Saad 1993), so x = Z y needs no final solve with M and a preconditioner that changes
between applications (inner CG to a tolerance) is allowed; restart length m = 30 and at most
300 iterations in total; orthogonalisation by CGS2; Givens rotations on the Hessenberg matrix.

``fgmres(apply_op, apply_prec, b, ...)``: apply_prec maps a basis vector to a direction z;
apply_op maps a direction z to A z in the space of b.  Directions may live in another space
than b (here: unscaled state increments versus scaled residuals).

Pins (tests/test_oracle_mg_krylov.py): exact solve for n <= m against numpy.linalg.solve, the
Arnoldi relation A Z_j = V_{j+1} H_j, orthonormality of V, monotone residual estimates that
equal the true residual.
"""
from __future__ import annotations

import numpy as np


def _givens(a, b):
    if b == 0.0:
        return 1.0, 0.0
    r = np.hypot(a, b)
    return a / r, b / r


def fgmres(apply_op, apply_prec, b, eta=1e-4, m=30, maxit=300, record=None):
    """Returns (x, info) with x = sum of y_j z_j over all cycles.

    info: dict(iters, converged, res_hist, arnoldi=[(V, Z, H)] per cycle when record).
    """
    bnorm = float(np.linalg.norm(b.ravel()))
    info = dict(iters=0, converged=False, res_hist=[bnorm])
    x = None
    if bnorm == 0.0:
        info["converged"] = True
        return np.zeros_like(apply_prec(np.zeros_like(b))), info
    target = eta * bnorm
    r = b.copy()
    total = 0
    while total < maxit:
        beta = float(np.linalg.norm(r.ravel()))
        if beta < target:
            info["converged"] = True
            break
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        Hraw = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        j_done = 0
        for j in range(m):
            z = apply_prec(V[j])
            Z.append(z)
            w = apply_op(z)
            h = np.zeros(j + 1)
            for _ in range(2):  # CGS2
                Vm = np.stack([v.ravel() for v in V])
                hh = Vm @ w.ravel()
                w = w - (hh @ Vm).reshape(w.shape)
                h += hh
            hn = float(np.linalg.norm(w.ravel()))
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            Hraw[:, j] = H[:, j]
            total += 1
            j_done = j + 1
            # apply previous rotations to the new column
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            res = abs(g[j + 1])
            info["res_hist"].append(res)
            if hn == 0.0 or res < target or total >= maxit:
                break
            V.append(w / hn)
        # solve the triangular system
        k = j_done
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        dx = sum(y[i] * Z[i] for i in range(k))
        x = dx if x is None else x + dx
        if record is not None:
            record.append(dict(V=V, Z=Z, y=y, H=Hraw[: k + 1, :k]))
        if abs(g[k]) < target:
            info["converged"] = True
            break
        if total >= maxit:
            break
        r = b - apply_op(x)
    info["iters"] = total
    if x is None:
        x = np.zeros_like(apply_prec(np.zeros_like(b)))
    return x, info
