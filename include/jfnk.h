/*
 * jfnk.h - C ABI of the MI355X (gfx950) implicit-step library.
 *
 * Jacobian-free Newton-Krylov solver with physics-based preconditioning for the inviscid
 * compressible equations with gravity and thermal conduction, after Viallet et al.,
 * "A Jacobian-free Newton-Krylov method for time-implicit multidimensional hydrodynamics"
 * (A&A 2016, arXiv 1512.03662).
 *
 * Conventions shared by every call
 * --------------------------------
 * State X and all vectors: contiguous FP64 structure-of-arrays in device memory,
 *   X[var][nz][ny][nx] (2D: X[var][ny][nx]), var = rho, e, u_x, u_y[, u_z]; x fastest.
 *   Cell (i,j,k) holds rho and e at its centre and u_d on its low-d face (Sect. 2: finite
 *   volumes with staggered velocities).  nvar = 2 + ndim, N = nx*ny[*nz], length nvar*N.
 * Ownership: array arguments belong to the caller; the library never keeps a pointer past
 *   the call.  The context owns its workspace, allocated by jfnk_create.
 * Space: every entry point works in unscaled physical variables; the diagonal scalings of
 *   the Newton system (Sect. 4.1, eq. jacobian_system_norm) are internal.
 * Wall-normal velocities on wall faces are stored and are zero; their residual row is
 *   rho_f u / dt - b (no flux acts on them) so J, M and J^T act there as the diagonal.
 * Streams: all work is ordered on the stream given to jfnk_create.  jfnk_residual,
 *   jfnk_jvp, jfnk_vjp and jfnk_vjp_prev are asynchronous; jfnk_precond_apply,
 *   jfnk_precond_apply_transpose, jfnk_implicit_step, jfnk_si_step, jfnk_adjoint_step and
 *   jfnk_cfl_dt synchronise the stream.
 * Errors: negative status codes; jfnk_last_error() gives the message.  Nothing throws
 *   across this boundary.  A context is not thread-safe; use one context per stream.
 */
#ifndef JFNK_H
#define JFNK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct jfnk_ctx jfnk_ctx;

enum {
  JFNK_OK = 0,
  JFNK_E_INVALID = -1,       /* bad argument, shape or option                          */
  JFNK_E_DEVICE = -2,        /* HIP error, including out-of-memory at create           */
  JFNK_E_NONFINITE = -3,     /* NaN/Inf met in a norm                                  */
  JFNK_E_GMRES_NOCONV = -4,  /* linear solve hit gmres_maxit (Newton continues)        */
  JFNK_E_NEWTON_NOCONV = -5, /* newton_max iterations without meeting newton_tol      */
  JFNK_E_INADMISSIBLE = -6   /* a Newton (or semi-implicit) update gives rho <= 0 or   *
                              * e <= 0; X holds that iterate (no line search, Sect. 4.1) */
};

enum { JFNK_BC_PERIODIC = 0, JFNK_BC_WALL = 1 };
enum { JFNK_CHI_NONE = 0, JFNK_CHI_CONST = 1, JFNK_CHI_POWER = 2 };
enum { JFNK_JV_FD = 0, JFNK_JV_EXACT = 1 };
enum { JFNK_PC_NONE = 0, JFNK_PC_SOUND = 1, JFNK_PC_SOUND_THERMAL = 2 };
enum { JFNK_FP64 = 0, JFNK_FP32 = 1 };

/* Problem: grid, equation of state, gravity and conductivity (Sect. 2, eqs. cons1-cons3,
 * chirad).  EOS with R = mu = 1 (Sect. 2, App. A): a_rad = 0 is the ideal gas
 * p = (gamma-1) rho e, T = (gamma-1) e; a_rad > 0 adds radiation in the diffusion limit,
 * p = rho T + a_rad T^4/3, e = T/(gamma-1) + a_rad T^4/rho (T(rho, e) by Newton's method,
 * Gamma1 and Gamma3 from the chain rule).                                              */
typedef struct {
  int32_t ndim;          /* 2 or 3                                                      */
  int32_t n[3];          /* cells along x, y, z (n[2] = 1 in 2D); each used axis >= 4  */
  double dx[3];          /* spacing per axis                                            */
  int32_t bc[3];         /* JFNK_BC_PERIODIC | JFNK_BC_WALL per axis                    */
  double gamma;          /* adiabatic index of the gas (Gamma1 = Gamma3 = gamma if ideal) */
  double g[3];           /* gravity vector                                              */
  int32_t chi_model;     /* NONE | CONST (chi0) | POWER (chi0 (T/chi_tref)^chi_exp)     */
  double chi0, chi_tref, chi_exp;
  double qwall[3][2];    /* prescribed conductive flux chi dT/dx_d on the low/high wall  */
  double theta;          /* time weighting: 1 = backward Euler, 1/2 = Crank-Nicolson    */
  double a_rad;          /* radiation constant (>= 0; 0: ideal gas)                     */
} jfnk_problem;

/* Solver options; jfnk_default_opts fills the values the paper uses (Sect. 4, 5.1.1).  */
typedef struct {
  double newton_tol;     /* ||R^-1 dX||_inf stopping threshold (eq. nr_terminate)       */
  int32_t newton_max;    /* maximum Newton iterations                                   */
  int32_t newton_min;    /* minimum Newton iterations (the paper enforces 2)            */
  int32_t gmres_m;       /* restart length (<= 70)                                       */
  int32_t gmres_maxit;   /* maximum GMRES iterations per Newton iteration               */
  double gmres_eta;      /* forcing term eta (eq. forcing_term)                         */
  int32_t jv_mode;       /* JFNK_JV_FD (eqs. jacobian_free, pert_old) | JFNK_JV_EXACT  */
  double fd_lambda;      /* lambda of eq. pert_old                                      */
  double alpha1, alpha2; /* velocity floors of the scalings (Sect. 4.1)                 */
  int32_t precond;       /* JFNK_PC_NONE | JFNK_PC_SOUND | JFNK_PC_SOUND_THERMAL        */
  int32_t ell_precision; /* JFNK_FP64 | JFNK_FP32 elliptic solves                       */
  double cg_eta;         /* parabolic-solve tolerance eta' (eq. forcing_term2)          */
  int32_t cg_maxit;      /* maximum CG iterations per elliptic solve; 0: the solve is    *
                          * one symmetric V-cycle, x = M b (a fixed linear operator, no   *
                          * CG step and no host synchronisation)                          */
  int32_t pc_schur;      /* 0: the paper's J~_V, which drops the velocity residual from  *
                          * the pressure equation (Sect. 3.3, delta form); 1: eliminate   *
                          * du exactly, keeping -dt div F~_u in the pressure right-hand  *
                          * side (exact inverse of J at a uniform state at rest without  *
                          * gravity or conduction)                                        */
  int32_t phase_timing;  /* 1: time the phases of a step with HIP events on the context's  *
                          * stream (jfnk_step_stats t_*); 0: no events (t_* = 0)          */
  int32_t mg_levels;     /* multigrid levels of the elliptic solves (Sect. 3.5 leaves the  *
                          * multi-level method's depth open): 0 = coarsen by 2 while every *
                          * used axis is even and longer than 4 cells; L >= 1 = at most L  *
                          * levels.  Fixed when the context is created (jfnk_set_opts      *
                          * rejects a change).  A coarsest level of more than 4096 cells   *
                          * is smoothed instead of solved exactly                          */
  int32_t mg_smooth;     /* degree k of the Chebyshev-Jacobi smoother on [0.5, 2] in       *
                          * D^-1 A, before and after the coarse correction: 1..8, 0 = 2    *
                          * (the default; its steps run fused with the V-cycle's other     *
                          * kernels, the other degrees one launch per step)                */
} jfnk_opts;

typedef struct {
  int32_t newton_its;    /* Newton iterations taken                                     */
  int32_t gmres_its;     /* GMRES iterations summed over Newton iterations              */
  int32_t cg_its;        /* CG iterations summed over all elliptic solves               */
  int32_t converged;     /* 1 if newton_tol was met                                     */
  double f0_norm;        /* ||L^-1 F(X^(0))||_2                                         */
  double f_norm;         /* ||L^-1 F|| at the last Newton iterate                       */
  double last_dx_norm;   /* ||R^-1 dX||_inf of the last correction                      */
  double dt;             /* time step used                                              */
  /* GPU time (ms, HIP events on the context's stream, host waits inside a phase included)
   * of the step's phases when opts.phase_timing = 1, else 0: the Newton residual with its
   * norms; the J.v products (FD: with the direction's norm); the preconditioner, its
   * set-up (elliptic coefficients, multigrid hierarchy, coarse inverse) included; the
   * Gram-Schmidt passes and normalisation of the Arnoldi vectors.                       */
  double t_resid, t_jv, t_prec, t_orth;
} jfnk_step_stats;

/* Fill *opts with the defaults: newton_tol 1e-8, newton_max 20, newton_min 2, gmres_m 30,
 * gmres_maxit 300, gmres_eta 1e-4, JV_FD, fd_lambda 1e-7, alpha1 1e-5, alpha2 1,
 * PC_SOUND, FP64, cg_eta 1e-4, cg_maxit 50, pc_schur 0, phase_timing 0.               */
void jfnk_default_opts(jfnk_opts* opts);

/* Create a context for one problem on one HIP stream (hip_stream: hipStream_t or NULL for
 * the null stream).  Allocates every workspace buffer.  JFNK_E_INVALID on a bad problem
 * or option, JFNK_E_DEVICE if allocation fails.  *out is NULL on failure.              */
int jfnk_create(const jfnk_problem* prob, const jfnk_opts* opts, void* hip_stream,
                jfnk_ctx** out);
int jfnk_destroy(jfnk_ctx* ctx);
/* Change solver options of an existing context (gmres_m may not exceed the created one). */
int jfnk_set_opts(jfnk_ctx* ctx, const jfnk_opts* opts);
size_t jfnk_workspace_bytes(const jfnk_ctx* ctx);
/* Message of the last error on ctx (or of the last failed jfnk_create if ctx is NULL).  */
const char* jfnk_last_error(const jfnk_ctx* ctx);

/* Store dt and b = U(X^n)/dt + (1-theta) R(X^n) (eq. crank_nicholson, theta-weighted)
 * for the next residual / jvp / vjp / precond calls.  X^n is copied.                   */
int jfnk_set_state_n(jfnk_ctx* ctx, const double* Xn, double dt);

/* F = U(X)/dt - theta R(X) - b (eq. crank_nicholson), R the staggered finite-volume
 * operator of Sect. 2 (van Leer upwind mass, energy and momentum fluxes, p div u,
 * conduction, gravity; ghost rules per axis: periodic wrap, or walls with even mirror and
 * zero wall-normal velocity).  Device pointers, FP64 SoA; async on the context's stream.
 * Needs jfnk_set_state_n.                                                              */
int jfnk_residual(jfnk_ctx* ctx, const double* X, double* F);

/* J v with J = dF/dX at X.  mode JFNK_JV_FD: (F(X + delta v) - F(X))/delta with
 * delta = lambda (lambda + ||R^-1 X||_2/||R^-1 v||_2) (eqs. jacobian_free, pert_old).
 * mode JFNK_JV_EXACT: forward-mode derivative of F (frozen upwind/limiter branches).   */
int jfnk_jvp(jfnk_ctx* ctx, const double* X, const double* v, double* Jv, int32_t mode);

/* J^T w at X (exact, frozen branches; deterministic gather form, no atomics).          */
int jfnk_vjp(jfnk_ctx* ctx, const double* X, const double* w, double* JTw);

/* (dF/dX^n)^T lam = -(dU/dX|_{X^n})^T lam / dt - (1-theta) (dR/dX|_{X^n})^T lam, the
 * dependence of the step residual on the previous state (eq. crank_nicholson).         */
int jfnk_vjp_prev(jfnk_ctx* ctx, const double* Xn, const double* lam, double* out);

/* z ~ +J^-1 r by the physics-based preconditioner frozen at X (Sect. 4.3 with the
 * semi-implicit schemes of Sects. 3.3-3.4); elliptic solves by multigrid-preconditioned
 * CG to opts.cg_eta in opts.ell_precision.  Needs jfnk_set_state_n (for dt).           */
int jfnk_precond_apply(jfnk_ctx* ctx, const double* X, const double* r, double* z);

/* z = M^-T w, the transpose of jfnk_precond_apply's operator at the same X (the adjoint
 * step's right preconditioner, unscaled): the transposed pointwise maps in reverse order
 * around the same symmetric elliptic solves.  Same arguments, requirements and
 * synchronisation as jfnk_precond_apply.                                                */
int jfnk_precond_apply_transpose(jfnk_ctx* ctx, const double* X, const double* w, double* z);

/* One implicit step: X holds X^n on entry and X^{n+1} on return (Sect. 4).  dt > 0 is
 * used as given.  Newton from X^n on the scaled system, FGMRES(m) with CGS2, J.v per
 * opts.jv_mode, right preconditioner per opts.precond.  Returns JFNK_OK when converged,
 * JFNK_E_NEWTON_NOCONV otherwise (X then holds the last iterate), JFNK_E_INADMISSIBLE when a
 * correction gives rho <= 0 or e <= 0 somewhere (X holds that iterate; the paper's Newton
 * iteration has no line search).  stats may be NULL.                                    */
int jfnk_implicit_step(jfnk_ctx* ctx, double* X, double dt, jfnk_step_stats* stats);

/* One step of the semi-implicit scheme used as a time stepper (Sect. 3.6): X holds X^n on
 * entry and X^{n+1} = X^n - M^-1 F(X^n) on return, F(X^n) = -R(X^n), M^-1 the physics-based
 * preconditioner of opts.precond (SOUND or SOUND_THERMAL; NONE is an error) frozen at X^n
 * with elliptic solves to opts.cg_eta.  opts.pc_schur = 1 gives the scheme derived in
 * Sect. 3.3 (Laplacian on p^{n+1}: implicit acoustics); 0 the delta-form J~_V applied to
 * (dV/dU) F.  Linear (no Newton), first order in time for theta = 1, stable only while the
 * advective CFL number stays small (the advection terms are explicit).  stats (may be NULL):
 * f0_norm = ||F(X^n)||_2, last_dx_norm = ||R^-1 dX||_inf, cg_its, converged = 1.         */
int jfnk_si_step(jfnk_ctx* ctx, double* X, double dt, jfnk_step_stats* stats);

/* Adjoint of one implicit step: given gbar_n1 = dL/dX^{n+1} at the converged X^{n+1} = Xn1
 * of the step from Xn with dt, solve J^T lam = gbar_n1 (FGMRES(m) on the scaled transposed
 * system R J^T L^-1, right preconditioner L M^-T R^-1 with the transposed physics-based
 * preconditioner, tolerance opts.gmres_eta) and return gbar_n = dL/dX^n =
 * -(dF/dX^n)^T lam.  Returns JFNK_E_GMRES_NOCONV (gbar_n still written) when the linear
 * solve stops at gmres_maxit.  dt is a constant of the step (not differentiated).       */
int jfnk_adjoint_step(jfnk_ctx* ctx, const double* Xn1, const double* Xn, double dt,
                      const double* gbar_n1, double* gbar_n, jfnk_step_stats* stats);

/* dt = cfl * min_d dx_d / max_c(|u_c| + c_s), u_c the cell-centred mean of the face
 * velocities (Introduction, CFL_hydro).  Synchronises; returns a negative value on error. */
double jfnk_cfl_dt(jfnk_ctx* ctx, const double* X, double cfl);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the time step of jfnk_cfl_dt without a
 * context.  *dt_out (device pointer, one double) receives cfl * min_d dx_d /
 * max_c(|u_c| + c_s) for the state X (device, FP64 SoA as everywhere) of problem prob; the
 * value is bit for bit the one jfnk_cfl_dt returns.  Asynchronous on hip_stream (NULL: the
 * null stream), whose device must be the current one.  Allocates nothing: the reduction's
 * block partials live in a static device array of 1024 doubles (8 KiB) that every device
 * the library runs on holds until the process ends; its address is looked up on the first
 * call on each device.  All calls on one device share that array, so calls that overlap
 * on one device (different streams, or threads) race.  JFNK_E_INVALID for a null pointer,
 * cfl <= 0, a problem jfnk_create would refuse, or a stream of another device (message in
 * jfnk_last_error(NULL)); JFNK_E_DEVICE on a HIP error.                                 */
int jfnk_cfl_dt_noalloc(const jfnk_problem* prob, const double* X, double cfl, double* dt_out,
                        void* hip_stream);

/* Measurement hooks (process-wide, not thread-safe).  jfnk_probe_enable(1) clears the
 * counters and from then on brackets every launch of the instrumented kernels with HIP
 * events on the stream it is launched on; jfnk_probe_enable(0) stops.  Kernel family k
 * (0 <= k < jfnk_probe_count(), name jfnk_probe_name(k)) reports through jfnk_probe_read
 * its summed event time in ms, its launch count, and the algorithmic bytes of those
 * launches (every field the kernel must read or write, counted once).  jfnk_probe_read
 * waits for the recorded events.                                                        */
int jfnk_probe_enable(int32_t on);
int jfnk_probe_count(void);
const char* jfnk_probe_name(int32_t k);
int jfnk_probe_read(int32_t k, double* ms, int64_t* launches, double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* JFNK_H */
