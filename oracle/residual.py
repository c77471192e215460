"""Oracle: staggered finite-volume residual of the time-discrete hydrodynamics system.

TEST INFRASTRUCTURE ONLY (see the package header).

Equations (Sect. 2, eqs. cons1-cons3): mass, internal energy with compressional work and
conduction div(chi grad T), momentum with gravity.  Unknowns X = (rho, e, u) and conserved
U = (rho, rho e, rho u) (Sect. 2).  Method of lines dU/dt = R_U(X) (eq. mol) and the
theta-weighted residual (eq. crank_nicholson gives theta = 1/2; theta = 1 is backward Euler):

    F(X) = U(X)/dt - theta R(X) - b,      b = U(X^n)/dt + (1 - theta) R(X^n).

The paper specifies the spatial scheme only as finite volumes with staggered velocities and
van Leer (1974) upwind monotone fluxes, second order and TVD (Sect. 2).  The stencil written
out here (the same reading is used by the GPU library):

* cells c = (i, j[, k]); rho, e at centres; u_d[c] on the low-d face of c.
* ghosts: periodic wrap; at walls scalars and tangential velocities mirror evenly,
  the wall-normal velocity is zero on both wall faces and odd outside.
* equation of state (oracle/eos.py), R = mu = 1: ideal gas p = (gamma-1) rho e,
  T = (gamma-1) e; with a_rad > 0 gas + radiation p = rho T + a T^4/3, e = c_v T + a T^4/rho.
* van Leer harmonic slope vl(a, b) = 2ab/(a+b) if ab > 0 else 0.
* upwind value at the low-d face of c by the sign of w (w >= 0 takes the left state):
  q_L = q[c-1] + vl(q[c-1]-q[c-2], q[c]-q[c-1])/2,  q_R = q[c] - vl(q[c]-q[c-1], q[c+1]-q[c])/2.
* mass flux f_d = u_d rho*, energy flux g_d = f_d e*, conductive flux
  q_d = chi_f (T[c]-T[c-1])/dx_d with chi_f the face mean (prescribed flux on wall faces).
* R_rho = -div f;  R_E = -div g - p div u + div q.
* momentum on the face control volume of u_d: Phi_dd at the cell centre carries u_d by the
  mean of the two adjacent mass fluxes, Phi_de on the (low-d, low-e) edge carries u_d along e
  by the mean of f_e of the two cells sharing that edge; upwind van Leer values of u_d;
  R_m,d = -ddiv Phi - (p[c]-p[c-1])/dx_d + rho_f g_d, rho_f the face mean of rho; zero on
  wall-normal wall faces (whose F row is therefore rho_f u / dt - b).

Every function is dtype-generic (float64 or complex128).  Branches are taken on the real
part and no abs() is applied, so ``Im F(X + i h v)/h`` is the exact frozen-branch J.v.

Pins: tests/test_oracle_residual.py (conservation, uniform states, hydrostatic balance,
mirror symmetry, linear acoustics dispersion through the exact step).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import eos

PERIODIC = "periodic"
WALL = "wall"
GHOST = 3


@dataclass
class Problem:
    shape: tuple          # cells per axis (nx, ny[, nz])
    dx: tuple             # spacing per axis
    bc: tuple             # 'periodic' | 'wall' per axis
    gamma: float
    g: tuple              # gravity per axis
    chi_model: str = "none"   # 'none' | 'const' | 'power'
    chi0: float = 0.0
    chi_tref: float = 1.0
    chi_exp: float = 3.0
    qwall: tuple = None   # per axis (lo, hi) prescribed chi dT/dx_d on wall faces
    theta: float = 1.0
    a_rad: float = 0.0    # radiation constant of the gas + radiation equation of state

    @property
    def nd(self):
        return len(self.shape)

    @property
    def nvar(self):
        return 2 + self.nd

    @property
    def field_shape(self):
        return tuple(reversed(self.shape))

    @property
    def ncell(self):
        return int(np.prod(self.shape))

    def axis(self, d):
        """numpy axis of spatial axis d in a single field array."""
        return self.nd - 1 - d

    @staticmethod
    def from_dict(p):
        nd = len(p["shape"])
        qwall = p.get("qwall") or ((0.0, 0.0),) * nd
        return Problem(shape=tuple(p["shape"]), dx=tuple(p["dx"]), bc=tuple(p["bc"]),
                       gamma=float(p["gamma"]), g=tuple(p.get("g") or (0.0,) * nd),
                       chi_model=p.get("chi_model", "none"), chi0=float(p.get("chi0", 0.0)),
                       chi_tref=float(p.get("chi_tref", 1.0)), chi_exp=float(p.get("chi_exp", 3.0)),
                       qwall=tuple(tuple(q) for q in qwall), theta=float(p.get("theta", 1.0)),
                       a_rad=float(p.get("a_rad", 0.0)))


def ghost_index(i, n, bc, odd_normal):
    """Map (possibly out-of-range) index i on an axis of n points to (source index, sign).

    Periodic: wrap.  Wall, cell-centred or tangential quantity: even mirror about the wall
    (i < 0 -> -1-i, i >= n -> 2n-1-i).  Wall-normal velocity on faces 0..n: zero on both wall
    faces (i = 0 and i = n), odd mirror outside (i < 0 -> -u[-i], i > n -> -u[2n-i]).
    """
    i = np.asarray(i)
    if bc == PERIODIC:
        return np.mod(i, n), np.ones(i.shape)
    if not odd_normal:
        src = np.where(i < 0, -1 - i, np.where(i >= n, 2 * n - 1 - i, i))
        return src, np.ones(i.shape)
    src = np.where(i < 0, -i, np.where(i > n, 2 * n - i, i))
    sign = np.where((i < 0) | (i > n), -1.0, np.where((i == 0) | (i == n), 0.0, 1.0))
    return np.clip(src, 0, n - 1), sign


class Stencil:
    """Evaluates cell quantities of X at offsets from a set of cells.

    ``cells`` is None (every cell, results shaped like a field) or a tuple of nd integer
    arrays of cell indices (ordered by axis d = 0..nd-1), results shaped like those arrays.
    """

    def __init__(self, prob: Problem, X, cells=None):
        self.prob = prob
        self.X = X
        nd = prob.nd
        if cells is None:
            coords = []
            for d in range(nd):
                shp = [1] * nd
                shp[prob.axis(d)] = prob.shape[d]
                coords.append(np.arange(prob.shape[d]).reshape(shp))
            self.coords = coords
        else:
            self.coords = [np.asarray(c) for c in cells]
        self._cache = {}

    # ---- raw gathers ---------------------------------------------------------------
    def gather(self, var, off):
        key = ("g", var, off)
        if key in self._cache:
            return self._cache[key]
        p = self.prob
        nd = p.nd
        srcs = [None] * nd
        sign = 1.0
        for d in range(nd):
            odd = (var == 2 + d) and p.bc[d] == WALL
            src, sg = ghost_index(self.coords[d] + off[d], p.shape[d], p.bc[d], odd)
            srcs[d] = src
            sign = sign * sg
        idx = tuple(srcs[d] for d in reversed(range(nd)))
        val = self.X[var][idx] * sign
        self._cache[key] = val
        return val

    def rho(self, off):
        return self.gather(0, off)

    def e(self, off):
        return self.gather(1, off)

    def u(self, d, off):
        return self.gather(2 + d, off)

    def p(self, off):
        return eos.pressure(self.prob, self.rho(off), self.e(off))

    def T(self, off):
        return eos.temperature(self.prob, self.rho(off), self.e(off))

    def chi(self, off):
        pr = self.prob
        if pr.chi_model == "none":
            return 0.0 * self.T(off)
        if pr.chi_model == "const":
            return pr.chi0 + 0.0 * self.T(off)
        return pr.chi0 * (self.T(off) / pr.chi_tref) ** pr.chi_exp

    def face_index(self, d, off):
        """Index (0..n_d) of the low-d face of cell c+off along d."""
        return self.coords[d] + off[d]


def sh(off, d, k):
    """Offset tuple moved by k along axis d."""
    o = list(off)
    o[d] += k
    return tuple(o)


def vl(a, b):
    """van Leer harmonic slope: 2ab/(a+b) when ab > 0, else 0 (branch on the real parts)."""
    mask = np.real(a) * np.real(b) > 0
    den = np.where(mask, a + b, 1.0)
    return np.where(mask, 2.0 * a * b / den, 0.0)


def upwind(qm2, qm1, q0, qp1, w):
    """Upwind van Leer value at the face between q[c-1] (qm1) and q[c] (q0); w >= 0 -> left."""
    qL = qm1 + 0.5 * vl(qm1 - qm2, q0 - qm1)
    qR = q0 - 0.5 * vl(q0 - qm1, qp1 - q0)
    return np.where(np.real(w) >= 0, qL, qR)


class Fluxes:
    """Face and edge fluxes of the staggered scheme, evaluated lazily with memoisation."""

    def __init__(self, st: Stencil):
        self.st = st
        self._c = {}

    def _memo(self, key, fn):
        if key not in self._c:
            self._c[key] = fn()
        return self._c[key]

    def recon_scalar(self, q, d, off, w):
        return upwind(q(sh(off, d, -2)), q(sh(off, d, -1)), q(off), q(sh(off, d, 1)), w)

    def mass(self, d, off):
        """f_d at the low-d face of c+off."""
        st = self.st

        def f():
            w = st.u(d, off)
            return w * self.recon_scalar(st.rho, d, off, w)
        return self._memo(("f", d, off), f)

    def energy(self, d, off):
        st = self.st

        def f():
            w = st.u(d, off)
            return self.mass(d, off) * self.recon_scalar(st.e, d, off, w)
        return self._memo(("g", d, off), f)

    def conduction(self, d, off):
        st = self.st
        pr = st.prob

        def f():
            chif = 0.5 * (st.chi(sh(off, d, -1)) + st.chi(off))
            q = chif * (st.T(off) - st.T(sh(off, d, -1))) / pr.dx[d]
            if pr.bc[d] == WALL and pr.chi_model != "none":
                fi = st.face_index(d, off)
                qlo, qhi = pr.qwall[d]
                q = np.where(fi == 0, qlo, np.where(fi == pr.shape[d], qhi, q))
            return q
        return self._memo(("q", d, off), f)

    def mom_centre(self, d, off):
        """Phi_dd at the centre of cell c+off: u_d carried along d."""
        st = self.st

        def f():
            m = 0.5 * (self.mass(d, off) + self.mass(d, sh(off, d, 1)))
            ustar = upwind(st.u(d, sh(off, d, -1)), st.u(d, off), st.u(d, sh(off, d, 1)),
                           st.u(d, sh(off, d, 2)), m)
            return m * ustar
        return self._memo(("Pc", d, off), f)

    def mom_edge(self, d, e, off):
        """Phi_de at the (low-d, low-e) edge of cell c+off: u_d carried along e."""
        st = self.st

        def f():
            m = 0.5 * (self.mass(e, sh(off, d, -1)) + self.mass(e, off))
            ustar = upwind(st.u(d, sh(off, e, -2)), st.u(d, sh(off, e, -1)), st.u(d, off),
                           st.u(d, sh(off, e, 1)), m)
            return m * ustar
        return self._memo(("Pe", d, e, off), f)


def _zero(nd):
    return (0,) * nd


def residual_R(prob: Problem, X, cells=None, with_abs=False):
    """Spatial operator R_U(X) (eq. mol) as an array shaped like X (or (nvar, K) for cells).

    With with_abs=True also returns A: per row the sum of the absolute values of the terms
    that make up R (used to normalise parity errors where R cancels to ~0).
    """
    st = Stencil(prob, X, cells)
    fl = Fluxes(st)
    nd = prob.nd
    o = _zero(nd)
    h = prob.dx
    R = [None] * prob.nvar
    A = [None] * prob.nvar
    ab = np.abs
    # mass
    acc, aacc = 0.0, 0.0
    for d in range(nd):
        t1 = fl.mass(d, sh(o, d, 1)) / h[d]
        t0 = fl.mass(d, o) / h[d]
        acc = acc - (t1 - t0)
        aacc = aacc + ab(t1) + ab(t0)
    R[0], A[0] = acc, aacc
    # internal energy
    acc, aacc = 0.0, 0.0
    divu = 0.0
    for d in range(nd):
        t1 = fl.energy(d, sh(o, d, 1)) / h[d]
        t0 = fl.energy(d, o) / h[d]
        acc = acc - (t1 - t0)
        aacc = aacc + ab(t1) + ab(t0)
        divu = divu + (st.u(d, sh(o, d, 1)) - st.u(d, o)) / h[d]
    pdiv = st.p(o) * divu
    acc = acc - pdiv
    aacc = aacc + ab(pdiv)
    if prob.chi_model != "none":
        for d in range(nd):
            t1 = fl.conduction(d, sh(o, d, 1)) / h[d]
            t0 = fl.conduction(d, o) / h[d]
            acc = acc + (t1 - t0)
            aacc = aacc + ab(t1) + ab(t0)
    R[1], A[1] = acc, aacc
    # momentum
    for d in range(nd):
        acc = -(fl.mom_centre(d, o) - fl.mom_centre(d, sh(o, d, -1))) / h[d]
        aacc = (ab(fl.mom_centre(d, o)) + ab(fl.mom_centre(d, sh(o, d, -1)))) / h[d]
        for e in range(nd):
            if e == d:
                continue
            t1 = fl.mom_edge(d, e, sh(o, e, 1)) / h[e]
            t0 = fl.mom_edge(d, e, o) / h[e]
            acc = acc - (t1 - t0)
            aacc = aacc + ab(t1) + ab(t0)
        gp = (st.p(o) - st.p(sh(o, d, -1))) / h[d]
        grav = 0.5 * (st.rho(sh(o, d, -1)) + st.rho(o)) * prob.g[d]
        acc = acc - gp + grav
        aacc = aacc + ab(st.p(o)) / h[d] + ab(st.p(sh(o, d, -1))) / h[d] + ab(grav)
        if prob.bc[d] == WALL:
            wall = st.coords[d] == 0
            acc = np.where(wall, 0.0, acc)
            aacc = np.where(wall, 0.0, aacc)
        R[2 + d], A[2 + d] = acc, aacc
    shape = np.broadcast(*[np.asarray(c) for c in st.coords]).shape
    R = np.stack([np.broadcast_to(r, shape) for r in R])
    if with_abs:
        A = np.stack([np.broadcast_to(np.real(a), shape) for a in A])
        return R, A
    return R


def conserved_U(prob: Problem, X, cells=None):
    """U(X) = (rho, rho e, rho_f u_d) with rho_f the face mean of rho (Sect. 2)."""
    st = Stencil(prob, X, cells)
    o = _zero(prob.nd)
    out = [st.rho(o), st.rho(o) * st.e(o)]
    for d in range(prob.nd):
        rf = 0.5 * (st.rho(sh(o, d, -1)) + st.rho(o))
        # the stored value of u_d is used (also on wall faces), not the ghost rule
        ud = _stored(st, 2 + d)
        out.append(rf * ud)
    shape = np.broadcast(*[np.asarray(c) for c in st.coords]).shape
    return np.stack([np.broadcast_to(v, shape) for v in out])


def _stored(st: Stencil, var):
    idx = tuple(np.asarray(st.coords[d]) for d in reversed(range(st.prob.nd)))
    return st.X[var][idx]


def rhs_b(prob: Problem, Xn, dt):
    """b = U(X^n)/dt + (1 - theta) R(X^n) (eq. crank_nicholson, theta-weighted)."""
    b = conserved_U(prob, Xn) / dt
    if prob.theta != 1.0:
        b = b + (1.0 - prob.theta) * residual_R(prob, Xn)
    return b


def residual_F(prob: Problem, X, b, dt, cells=None):
    """F(X) = U(X)/dt - theta R(X) - b (eq. crank_nicholson with theta-weighting)."""
    U = conserved_U(prob, X, cells)
    R = residual_R(prob, X, cells)
    if cells is not None:
        idx = tuple(np.asarray(cells[d]) for d in reversed(range(prob.nd)))
        bb = np.stack([b[k][idx] for k in range(prob.nvar)])
    else:
        bb = b
    return U / dt - prob.theta * R - bb


def residual_scale(prob: Problem, X, b, dt):
    """Per-variable magnitude S_k used to normalise residual parity errors.

    S_k = max_c(|U_k(X)|/dt + |b_k|) + max_c A_k, with A_k the sum of absolute terms of R.
    """
    U = conserved_U(prob, X)
    _, A = residual_R(prob, X, with_abs=True)
    nv = prob.nvar
    S = np.empty(nv)
    for k in range(nv):
        S[k] = np.max(np.abs(U[k]) / dt + np.abs(b[k])) + np.max(A[k])
    return S


def cfl_dt(prob: Problem, X, cfl):
    """dt = cfl * min_d dx_d / max_c(|u_c| + c_s), u_c the face-to-centre mean (Introduction)."""
    st = Stencil(prob, X)
    o = _zero(prob.nd)
    u2 = 0.0
    for d in range(prob.nd):
        uc = 0.5 * (st.u(d, o) + st.u(d, sh(o, d, 1)))
        u2 = u2 + uc * uc
    cs = eos.sound_speed(prob, st.rho(o), st.e(o))
    return cfl * min(prob.dx) / float(np.max(np.sqrt(u2) + cs))
