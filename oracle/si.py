"""Oracle: the semi-implicit scheme as a stand-alone time stepper (Sect. 3.6).

TEST INFRASTRUCTURE ONLY (see the package header).

The five steps of Sect. 3.6: F_U(X^n) = -R_U(X^n); transform F_U to the primitive variables
(dV/dU); solve the semi-implicit system J~_V dV = -F~_V; transform dV back (dX/dV);
X^{n+1} = X^n + dX.  Steps 2-4 are the physics-based preconditioner applied to F_U
(``oracle/pbp.py``, which returns z ~ +J^-1 r), so X^{n+1} = X^n - M^-1 F_U(X^n).

Reading of the system solved in step 3.  The scheme derived in Sect. 3.3 puts the Laplacian
on p^{n+1} (the pressure equation after u^{n+1} = u^n - dt(...)^n - dt grad p^{n+1}/rho is
substituted into the divergence): in delta form that is the Schur-complement elimination,
which keeps -dt div F~_u in the pressure right-hand side (``schur=True``, the default).  The
delta-form matrix J~_V of Sect. 3.3, used with F~_V = (dV/dU) F_U literally, drops that term
(``schur=False``): from a state at rest its first step leaves p and e unchanged and moves u
by the explicit pressure force.  Both are linear in dX (Picard linearisation, Sect. 3.6) and
first order in time; theta < 1 uses the theta-weighted preconditioner (tau = theta dt).

Pins (tests/test_oracle_si.py): at a uniform state at rest the Schur form advances a small
standing sound wave by the closed-form theta-step factor; the J~_V form's first step from
rest is the explicit momentum update with p, e unchanged; wall-normal wall velocities stay 0.
"""
from __future__ import annotations

from .pbp import PBP
from .residual import Problem, residual_F, rhs_b


def si_step(prob: Problem, Xn, dt, mode="sound", schur=True, solver_factory=None):
    """X^{n+1} of one semi-implicit step from X^n (direct elliptic solves by default)."""
    F = residual_F(prob, Xn, rhs_b(prob, Xn, dt), dt)  # = -R(X^n) for every theta
    z = PBP(prob, Xn, dt, mode, solver_factory=solver_factory, schur=schur).apply(F)
    return Xn - z
