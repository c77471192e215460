"""Plain, slow CPU FP64 oracle of the JFNK + physics-based-preconditioner implicit step.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark may import this package; the GPU library never calls into it and shares no
code with it.

Written from Viallet et al. 2016 (A&A, arXiv 1512.03662), "A Jacobian-free Newton-Krylov
method for time-implicit multidimensional hydrodynamics":

* ``residual``  - conservation laws (Sect. 2, eqs. cons1-cons3), conductivity (eq. chirad),
                  method of lines and the time-discrete residual (eqs. mol, crank_nicholson)
                  with a theta-weighting; the staggered finite-volume van Leer discretisation
                  the paper only names (Sect. 2) is written out in the module docstring.
* ``scaling``   - diagonal scalings L and R (Sect. 4.1, eq. jacobian_system_norm).
* ``jacobian``  - finite-difference J.v (Sect. 4.2, eqs. jacobian_free, pert_old), exact J.v
                  by the complex step, coloured sparse Jacobian.
* ``pbp``       - transformation matrices (Sect. 3.2, App. B), semi-implicit sound-wave and
                  thermal-diffusion schemes (Sects. 3.3-3.4) used as preconditioner
                  (Sect. 4.3) with direct sparse elliptic solves.
* ``mg``        - multigrid-preconditioned CG for the parabolic systems (Sect. 3.5 replaces
                  GMRES + smoothed aggregation by this), FP64 or emulated FP32.
* ``krylov``    - right-preconditioned flexible GMRES(m) with CGS2 (Sects. 4.1, 4.3).
* ``newton``    - inexact Newton on the scaled system (Sect. 4.1) and exact Newton with a
                  sparse LU solve (the plain definition of the step's root).
* ``adjoint``   - transposed step for gradients through implicit steps.

Parity status of each function is stated in its module header.
"""
