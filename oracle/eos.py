"""Oracle: equation of state.

TEST INFRASTRUCTURE ONLY (see the package header).

The system of Sect. 2 is closed by an equation of state; units with R = mu = 1.

* ideal gas (a_rad = 0): p = (gamma - 1) rho e, T = (gamma - 1) e, Gamma1 = Gamma3 = gamma;
* gas + radiation in the diffusion limit (Sect. 2; a_rad > 0, the radiation constant in these
  units): p = rho T + a T^4 / 3, e = c_v T + a T^4 / rho with c_v = 1/(gamma - 1).  T(rho, e)
  is the positive root of c_v T + a T^4/rho - e, increasing and convex in T; Newton's method
  from min((gamma - 1) e, (rho e / a)^(1/4)), which lies above the root (by at most 38%),
  decreases to it quadratically; NEWTON_ITS = 12 steps leave it at rounding.

Derivatives used by the preconditioner's transforms (App. A): dp/drho|_e and dp/de|_rho from
the chain rule through T(rho, e); Gamma1 = (rho/p)(dp/drho|_e + p/rho^2 dp/de|_rho) (the
adiabatic sound speed c_s^2 = Gamma1 p / rho); Gamma3 - 1 = dp/de|_rho / rho, so that
dp/drho|_e = (p/rho)(Gamma1 - Gamma3 + 1) and dp/de|_rho = rho (Gamma3 - 1) as the paper
writes them.  c_v here is de/dT|_rho (the thermal preconditioner's dT = de / c_v).

Every function is holomorphic in (rho, e) (complex steps pass through the Newton iteration;
branch decisions use real parts).

Pins (tests/test_oracle_eos.py): a_rad = 0 reproduces the ideal gas exactly; T(rho, e) inverts
e(rho, T) to roundoff; Gamma1 and Gamma3 match the closed forms of a gas-radiation mixture in
terms of beta = p_gas / p (Chandrasekhar); the derivatives match complex steps of p(rho, e).
"""
from __future__ import annotations

import numpy as np

NEWTON_ITS = 12


def temperature(prob, rho, e):
    if prob.a_rad == 0.0:
        return (prob.gamma - 1.0) * e
    cv = 1.0 / (prob.gamma - 1.0)
    a = prob.a_rad
    t1 = e / cv
    t2 = (rho * e / a) ** 0.25
    T = np.where(np.real(t1) < np.real(t2), t1, t2)
    for _ in range(NEWTON_ITS):
        f = cv * T + a * T ** 4 / rho - e
        T = T - f / (cv + 4.0 * a * T ** 3 / rho)
    return T


def pressure(prob, rho, e):
    if prob.a_rad == 0.0:
        return (prob.gamma - 1.0) * rho * e
    T = temperature(prob, rho, e)
    return rho * T + prob.a_rad * T ** 4 / 3.0


def thermo(prob, rho, e):
    """(p, T, dp/drho|_e, dp/de|_rho, Gamma1, c_v = de/dT|_rho) at each cell."""
    g = prob.gamma
    if prob.a_rad == 0.0:
        p = (g - 1.0) * rho * e
        T = (g - 1.0) * e
        return p, T, (g - 1.0) * e, (g - 1.0) * rho, g + 0.0 * rho, 1.0 / (g - 1.0) + 0.0 * rho
    a = prob.a_rad
    cv = 1.0 / (g - 1.0)
    T = temperature(prob, rho, e)
    p = rho * T + a * T ** 4 / 3.0
    eT = cv + 4.0 * a * T ** 3 / rho          # de/dT|_rho
    erho = -a * T ** 4 / rho ** 2             # de/drho|_T
    pT = rho + 4.0 * a * T ** 3 / 3.0         # dp/dT|_rho
    prho = T                                  # dp/drho|_T
    dTde = 1.0 / eT
    dTdr = -erho / eT
    dpde = pT * dTde
    dpdr = prho + pT * dTdr
    G1 = (rho / p) * (dpdr + p / rho ** 2 * dpde)
    return p, T, dpdr, dpde, G1, eT


def sound_speed(prob, rho, e):
    if prob.a_rad == 0.0:
        return np.sqrt(prob.gamma * (prob.gamma - 1.0) * e)
    p, _, dpdr, dpde, _, _ = thermo(prob, rho, e)
    return np.sqrt(dpdr + p / rho ** 2 * dpde)
