"""Oracle: diagonal scalings of the Newton system (Sect. 4.1, eq. jacobian_system_norm).

TEST INFRASTRUCTURE ONLY.

L (residual scaling) and R (unknown scaling), per cell and variable:
  L_rho = rho, L_E = rho e, L_u = rho_f max(|u|, alpha1 c_s,f)
  R_rho = rho, R_e = e,     R_u = max(|u|, alpha2 c_s,f)
with the face means rho_f, c_s,f of the two cells sharing the face (mirror ghost at walls),
u the stored face velocity.  Default alpha1 = 1e-5, alpha2 = 1 (Sect. 4.1 / Sect. 5.1.1).

Pinned by tests/test_oracle_scaling_pbp.py against the definitions on hand-built states.
"""
from __future__ import annotations

import numpy as np

from . import eos

from .residual import Problem, Stencil, sh


def scaling_LR(prob: Problem, X, alpha1=1e-5, alpha2=1.0):
    st = Stencil(prob, X)
    nd = prob.nd
    o = (0,) * nd
    rho = st.rho(o)
    e = st.e(o)
    L = np.empty_like(X)
    R = np.empty_like(X)
    L[0] = rho
    L[1] = rho * e
    R[0] = rho
    R[1] = e
    cs = lambda off: eos.sound_speed(prob, st.rho(off), st.e(off))
    for d in range(nd):
        csf = 0.5 * (cs(sh(o, d, -1)) + cs(o))
        rf = 0.5 * (st.rho(sh(o, d, -1)) + rho)
        au = np.abs(X[2 + d])
        L[2 + d] = rf * np.maximum(au, alpha1 * csf)
        R[2 + d] = np.maximum(au, alpha2 * csf)
    return L, R
