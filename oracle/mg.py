"""Oracle: geometric multigrid-preconditioned conjugate gradients for the parabolic systems.

TEST INFRASTRUCTURE ONLY.

The paper solves its parabolic systems with a Krylov method preconditioned by a multi-level
method, stopped at ||P x - b||_2 < eta' ||b||_2 with eta' = 1e-4, and replaces random
eigenvalue estimates by a norm bound so that restarts reproduce (Sect. 3.5).  Because the
operators here are SPD (see ``pbp``), CG is used with one symmetric V-cycle as
preconditioner:

* cell-centred coarsening by 2 per axis while every axis is even and longer than 4 cells,
  and, when ``max_levels`` > 0, while there are fewer than ``max_levels`` levels (the paper
  leaves the multi-level method's depth open);
* coarse diagonal = mean of the 2^d children; coarse face weight = mean of the covered fine
  face weights / 4 (the same operator rediscretised at twice the spacing);
* restriction = mean of the children; prolongation = piecewise-constant injection;
* smoother: Chebyshev polynomial of degree k (default 2) in D^-1 A on [lmax/4, lmax] with
  lmax = 2, the Gershgorin bound of D^-1 A (discs centred at 1 with radius < 1), by the
  three-term recurrence of the Chebyshev semi-iteration; the same smoother before and after
  the coarse correction keeps the V-cycle symmetric;
* coarsest level: dense Cholesky (always in FP64) while it has at most ``DENSE_MAX`` = 4096
  cells.  A grid with an odd axis cannot be coarsened that far (for example the 72 x 65 x 65
  grid of the paper's 3D red-giant run, Sect. 5.2); its coarsest level is then not solved
  but smoothed: the same Chebyshev smoothing from zero, then again from that iterate (the
  polynomial of D^-1 A applied twice keeps the V-cycle symmetric positive definite).

``dtype=np.float32`` emulates the mixed-precision variant: coefficients, vectors and dot
products in FP32, the right-hand side divided by its FP64 2-norm before the cast, the
result cast back and rescaled.

Pins (tests/test_oracle_mg_krylov.py): the V-cycle is a symmetric positive definite operator
(dense check on small grids); PCG meets its stopping rule and agrees with the sparse direct
solve within eta' times the condition-number bound; iteration counts stay bounded as the grid
is refined.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .pbp import EllOp, _roll, _wall_slice
from .residual import Problem, WALL


def coarsen_shape(shape):
    if all(n % 2 == 0 and n > 4 for n in shape):
        return tuple(n // 2 for n in shape)
    return None


def _restrict_mean(prob, a):
    """Mean over the 2^d children of each coarse cell."""
    out = a
    for d in range(prob.nd):
        ax = prob.axis(d)
        sl0 = [slice(None)] * prob.nd
        sl1 = [slice(None)] * prob.nd
        sl0[ax] = slice(0, None, 2)
        sl1[ax] = slice(1, None, 2)
        out = 0.5 * (out[tuple(sl0)] + out[tuple(sl1)])
    return out


def _prolong(prob_f, a):
    out = a
    for d in range(prob_f.nd):
        out = np.repeat(out, 2, axis=prob_f.axis(d))
    return out


def _coarse_face_weights(prob_f, w_f, d):
    """Coarse low-d face weights: mean of the fine faces covered, divided by 4."""
    ax = prob_f.axis(d)
    sl = [slice(None)] * prob_f.nd
    sl[ax] = slice(0, None, 2)  # fine faces that coincide with coarse faces
    w = w_f[tuple(sl)]
    # average over the transverse children
    for e in range(prob_f.nd):
        if e == d:
            continue
        axe = prob_f.axis(e)
        s0 = [slice(None)] * prob_f.nd
        s1 = [slice(None)] * prob_f.nd
        s0[axe] = slice(0, None, 2)
        s1[axe] = slice(1, None, 2)
        w = 0.5 * (w[tuple(s0)] + w[tuple(s1)])
    return w / 4.0


class Level:
    def __init__(self, prob: Problem, op: EllOp):
        self.prob = prob
        self.op = op
        self.dinv = op.dinv()


class Multigrid:
    LMAX = 2.0
    LMIN = 0.5
    DENSE_MAX = 4096

    def __init__(self, op: EllOp, dtype=np.float64, max_levels=0, degree=2):
        self.dtype = dtype
        self.degree = degree
        prob = op.prob
        cast = lambda a: np.asarray(a, dtype=dtype)
        self.levels = [Level(prob, EllOp(prob, cast(op.diag), [cast(w) for w in op.w]))]
        while max_levels == 0 or len(self.levels) < max_levels:
            cur = self.levels[-1]
            cs = coarsen_shape(cur.prob.shape)
            if cs is None:
                break
            pc = Problem(shape=cs, dx=tuple(2 * h for h in cur.prob.dx), bc=cur.prob.bc,
                         gamma=cur.prob.gamma, g=cur.prob.g)
            diag_c = _restrict_mean(cur.prob, cur.op.diag)
            w_c = [_coarse_face_weights(cur.prob, cur.op.w[d], d) for d in range(cur.prob.nd)]
            self.levels.append(Level(pc, EllOp(pc, diag_c.astype(dtype), [w.astype(dtype) for w in w_c])))
        coarse = self.levels[-1]
        self.coarse_chol = None
        if coarse.prob.ncell <= self.DENSE_MAX:
            A = coarse.op.to_sparse().toarray().astype(np.float64)
            self.coarse_chol = sla.cho_factor(A, lower=True)

    def smooth(self, lev: Level, b, x):
        """Chebyshev-Jacobi smoothing of A x = b starting from x: d_0 = D^-1 r_0 / theta,
        then d_i = rho_i rho_{i-1} d_{i-1} + (2 rho_i / delta) D^-1 r_i with
        rho_0 = delta / theta, rho_i = 1 / (2 theta / delta - rho_{i-1}); x += d_i each step."""
        t = self.dtype
        theta = t(0.5 * (self.LMAX + self.LMIN))
        delta = t(0.5 * (self.LMAX - self.LMIN))
        sigma = theta / delta
        rho = t(1.0) / sigma
        r = b - lev.op.apply(x)
        dvec = lev.dinv * r / theta
        x = x + dvec
        for _ in range(1, self.degree):
            r = b - lev.op.apply(x)
            rho_new = t(1.0) / (t(2.0) * sigma - rho)
            dvec = rho_new * rho * dvec + (t(2.0) * rho_new / delta) * (lev.dinv * r)
            rho = rho_new
            x = x + dvec
        return x

    def vcycle(self, b, level=0):
        lev = self.levels[level]
        if level == len(self.levels) - 1:
            if self.coarse_chol is None:  # too large for the dense solve: smoothing only
                return self.smooth(lev, b, self.smooth(lev, b, np.zeros_like(b)))
            x = sla.cho_solve(self.coarse_chol, b.ravel().astype(np.float64))
            return x.reshape(b.shape).astype(self.dtype)
        x = self.smooth(lev, b, np.zeros_like(b))
        r = b - lev.op.apply(x)
        xc = self.vcycle(_restrict_mean(lev.prob, r), level + 1)
        x = x + _prolong(lev.prob, xc)
        return self.smooth(lev, b, x)


def pcg(op: EllOp, b, eta=1e-4, maxit=50, dtype=np.float64, mg=None, stats=None):
    """CG on A x = b preconditioned by one V-cycle; stop when ||r||_2 < eta ||b||_2.

    Returns x in float64.  With dtype=float32, b is divided by ||b||_2 (FP64) before the
    cast and the result multiplied back.  maxit = 0: the solve is the preconditioning
    V-cycle alone, x = M b (a fixed, symmetric linear operator; no CG step).
    """
    if mg is None:
        mg = Multigrid(op, dtype)
    A = mg.levels[0].op
    bnorm64 = float(np.linalg.norm(b.ravel()))
    if bnorm64 == 0.0:
        if stats is not None:
            stats.append(0)
        return np.zeros(b.shape)
    if dtype == np.float32:
        bb = (b / bnorm64).astype(np.float32)
    else:
        bb = b.astype(np.float64)
    dot = lambda u, v: np.dot(u.ravel(), v.ravel())
    x = np.zeros_like(bb)
    r = bb.copy()
    bn = np.sqrt(dot(bb, bb))
    z = mg.vcycle(r)
    if maxit == 0:
        x = z
    p = z.copy()
    rz = dot(r, z)
    it = 0
    for it in range(1, maxit + 1):
        Ap = A.apply(p)
        alpha = rz / dot(p, Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        if np.sqrt(dot(r, r)) < eta * bn:
            break
        z = mg.vcycle(r)
        rz_new = dot(r, z)
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    if stats is not None:
        stats.append(it)
    x = x.astype(np.float64)
    if dtype == np.float32:
        x = x * bnorm64
    return x


class PCGSolver:
    """Callable b -> A^-1 b by MG-preconditioned CG (for ``pbp.PBP(solver_factory=...)``)."""

    def __init__(self, op, eta=1e-4, maxit=50, dtype=np.float64, max_levels=0, degree=2):
        self.op = op
        self.eta, self.maxit, self.dtype = eta, maxit, dtype
        self.mg = Multigrid(op, dtype, max_levels, degree)
        self.iters = []

    def __call__(self, b):
        return pcg(self.op, b, self.eta, self.maxit, self.dtype, self.mg, self.iters)

    @staticmethod
    def factory(eta=1e-4, maxit=50, dtype=np.float64, max_levels=0, degree=2):
        return lambda op: PCGSolver(op, eta, maxit, dtype, max_levels, degree)
