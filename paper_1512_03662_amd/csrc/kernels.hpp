// Host-callable launchers of the device kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "common.hpp"

namespace jfnk {

struct ResidArgs {
  const double* X = nullptr;         // state
  const double* V = nullptr;         // direction (tangent or finite-difference step)
  const double* B = nullptr;         // subtracted vector (b, or G0 for finite differences)
  double* out = nullptr;
  double* G0 = nullptr;              // optional second output cU U + cR R (value mode)
  double cU = 0.0, cR = 0.0;         // out = cU U + cR R - B
  const double* fd_norms = nullptr;  // device [||R^-1 X||^2, ||R^-1 V||^2] (FD mode)
  double fd_lambda = 1e-7;
  double* shift = nullptr;           // FD mode: state-sized scratch for X + delta V, or null
  int scaleL = 0;                    // divide each row by L
  double alpha1 = 1e-5;
};

// mode 0: value, 1: exact tangent (forward mode), 2: finite difference
void launch_resid(const Grid& G, const ResidArgs& a, int mode, hipStream_t s);
// which 0: L (alpha = alpha1), 1: R (alpha = alpha2); mode 0: out = in/S, 1: out = in*S
void launch_scale_LR(const Grid& G, const double* X, double alpha, int which, const double* in,
                     double* out, int mode, hipStream_t s);

// ---- deterministic reductions ---------------------------------------------------------
constexpr int kRedBlocks = 1024;   // maximum blocks of a reduction grid
constexpr int kMaxK = 72;          // maximum simultaneous sums (Krylov basis size + 1)

struct RedWS {
  double* part = nullptr;          // kRedBlocks * 2 kMaxK partials
  unsigned int* count = nullptr;   // unused (kept zero)
};

// out[k] = sum over b < nb of part[b*K + k], in block order (one block)
void launch_finalize_sum(const RedWS& ws, int nb, int K, double* out, hipStream_t s);

template <class T>
void launch_dot(size_t n, const T* a, const T* b, double* out, const RedWS& w, hipStream_t s);
// Arnoldi orthogonalisation with delayed reorthogonalisation (slots 0..K-2 of V final, slot
// K-1 the newest vector after one pass, w the new product):
// sums[k] = V_k . V_{K-1}, sums[K + k] = V_k . w for k < K
void launch_dcgs2_dots(size_t n, const double* V, size_t ld, int K, const double* w, double* sums,
                       const RedWS& ws, hipStream_t s, const double* qn2 = nullptr);
// slot K-1 reorthogonalised and renormalised (K >= 2), dst = w orthogonalised against slots
// 0..K-1, *nrm2 = ||dst||^2 (coefficients formed on the device from sums)
void launch_dcgs2_update(size_t n, double* V, size_t ld, int K, const double* sums, const double* w, double* dst,
                         double* nrm2, const RedWS& ws, hipStream_t s, const double* qn2 = nullptr);
// (qn2: slot K-1 is kept unnormalised and read as V_{K-1} / sqrt(*qn2); the update pass writes
// it back normalised)
// dst = src / sqrt(*nrm2)
void launch_scale_by_inv_sqrt(size_t n, const double* src, const double* nrm2, double* dst,
                              hipStream_t s);
// dst = sum_k y[k] Z_k (y on the device)
void launch_lincomb(size_t n, const double* Z, size_t ld, int K, const double* y, double* dst,
                    hipStream_t s);
// y = a x + y, x and y double
void launch_axpy(size_t n, double a, const double* x, double* y, hipStream_t s);
void launch_fill(size_t n, double v, double* y, hipStream_t s);
template <class T>
void launch_fill_t(size_t n, T v, T* y, hipStream_t s);

// scaled norm of a state-shaped vector: out = sum (V/R(X))^2
void launch_scaled_norm2(const Grid& G, const double* X, const double* V, double alpha2,
                         double* out, const RedWS& ws, hipStream_t s);
// out[0] = max |V/R(X)|, out[1] = max -min(rho, e) of X + sgn V (negative: admissible)
void launch_newton_check(const Grid& G, const double* X, const double* V, double alpha2, double sgn,
                         double* out, const RedWS& ws, hipStream_t s);
// max over cells of |u_c| + c_s (CFL)
void launch_cfl_speed(const Grid& G, const double* X, double* out, const RedWS& ws, hipStream_t s);
// *dt = num / max_c(|u_c| + c_s) on the device, with cfl_partials(G) block partials in part
int cfl_partials(const Grid& G);
void launch_cfl_dt_dev(const Grid& G, const double* X, double num, double* part, double* dt, hipStream_t s);

// ---- physics-based preconditioner ------------------------------------------------------
struct Level {              // one multigrid level of one elliptic operator
  int n[3];
  int N;
  int stride[3];
  void* diag = nullptr;     // T[N]
  void* w[3] = {nullptr, nullptr, nullptr};  // T[N] low-face weights per axis
  void* dinv = nullptr;     // T[N]
  void* b = nullptr;        // T[N] right-hand side / restricted residual
  void* x = nullptr;        // T[N] solution
  void* t1 = nullptr;       // T[N]
  void* t2 = nullptr;       // T[N]
};

// pressure (op 0) and thermal (op 1) coefficients on the finest level, FP64
void launch_ell_coef(const Grid& G, const double* X, double dt, int op, double* diag,
                     double* const* w, hipStream_t s);
template <class T>
void launch_ell_coarsen(const Grid& G, const Level& f, const Level& c, hipStream_t s);
template <class T>
void launch_ell_dinv(const Grid& G, const Level& L, hipStream_t s);
void launch_level_to_f32(const Level& src, const Level& dst, int nd, hipStream_t s);

// ---- multigrid-preconditioned CG driven from the device --------------------------------
// Control block of one CG solve (device memory).  Every kernel of an iteration returns at
// once when flag != 0, so the host may enqueue iterations ahead of the convergence test.
struct CGCtl {
  double rz[2];   // (r, z) of the last two iterations, slot = iteration & 1
  double bb;      // ||b||^2
  double rr;      // ||r||^2 after the last update
  int flag;       // 0 running, 1 stopped (converged or iteration limit), -1 non-finite
  int its;        // iterations of the stopped solve
};
// partial sums, kRedBlocks doubles each: (b,b), (r,z), (p,q), (r,r)
enum { kPartBB = 0, kPartRZ = 1, kPartPQ = 2, kPartRR = 3, kPartCount = 4 };
struct CGArgs {
  CGCtl* ctl = nullptr;
  double* part = nullptr;   // kPartCount * kRedBlocks
  int np = 0;               // partials per sum (cg_partials(N) of level 0)
  double eta = 1e-4;        // stop when ||r|| < eta ||b||
  int maxit = 50;
};
int cg_partials(size_t n);

// V-cycle pieces.  presmooth with init: first smoothing of a solve (resets the control block,
// writes the (b, b) partials); restrict with conv_it > 0: also the convergence decision of
// that iteration; smooth2 with rz: also the (b, x) partials.
template <class T>
void launch_mg_presmooth(const Grid& G, const Level& L, const T* b, T* x, const CGArgs& g, bool init,
                         hipStream_t s);
template <class T>
void launch_mg_restrict_resid(const Grid& G, const Level& f, const T* b, const T* x, T* bc,
                              const Level& c, const CGArgs& g, int conv_it, hipStream_t s);
template <class T>
void launch_mg_prolong_smooth1(const Grid& G, const Level& f, const T* b, const T* x2, const T* xc,
                               const Level& c, T* x1, T* d0, const CGArgs& g, hipStream_t s);
template <class T>
void launch_mg_smooth2(const Grid& G, const Level& L, const T* b, const T* x1, const T* d0, T* x,
                       const CGArgs& g, bool rz, hipStream_t s);
template <class T>
void launch_dense_matvec(int n, const double* A, const T* x, T* y, const CGArgs& g, hipStream_t s);
// Chebyshev-Jacobi smoothing of any degree, one launch per step (the fused V-cycle kernels
// implement degree 2): coefficients c1[i], c2[i] of steps i = 1..k-1; the first step from
// zero (x = d = D^-1 b / theta); a further step (d = c1 d + c2 D^-1 (b - A xin),
// xout = xin + d; xout != xin)
void cheb_coefs(int k, double* c1, double* c2);
template <class T>
void launch_cheb_zero(const Grid& G, const Level& L, const T* b, T* x, T* d, const CGArgs& g, hipStream_t s);
template <class T>
void launch_cheb_step(const Grid& G, const Level& L, const T* b, const T* xin, T* xout, T* d, double c1, double c2,
                      const CGArgs& g, hipStream_t s);

// coarse part of a V-cycle (levels of at most kCoarseMaxN cells) in one workgroup
constexpr int kCoarseMaxN = 1024;
constexpr int kCoarseThreads = 1024;
constexpr int kMaxLevels = 12;
enum { kCoarseInit = 1, kCoarseConv = 2, kCoarseRZ = 4, kCoarseFromPre = 8, kCoarseToUp = 16 };
struct CoarseArgs {
  int nl, tot;
  int n[kMaxLevels][3], stride[kMaxLevels][3], N[kMaxLevels], off[kMaxLevels];
  int coff[kMaxLevels];  // offset of the level's coefficients in LDS, -1: read from memory
  int bc[3];
  const void* diag[kMaxLevels];
  const void* w[kMaxLevels][3];
  const void* dinv[kMaxLevels];
  const double* Ainv;   // dense inverse of the last level
  const void* b0;       // right-hand side of the first fused level
  void* x0;             // its iterate: in with kCoarseFromPre, out unless kCoarseToUp
  void* t1_0;           // out with kCoarseToUp: first post-smoothing step of the first level
  void* t2_0;
};
template <class T>
void launch_vcycle_coarse(const Grid& G, const Level* lv, int nl, const double* Ainv, const T* b0,
                          T* x0, const CGArgs& g, int mode, int it, hipStream_t s);
// largest coarse level of a fused level pair
constexpr int kFusePairMaxN = 65536;
// fused level pairs: restriction f -> c with the first smoothing of c (conv_it > 0: also the
// convergence decision); second smoothing of c with the prolongation to f and f's first
// post-smoothing step
template <class T>
void launch_mg_down(const Grid& G, const Level& f, const T* bf, const T* xf, const Level& c, T* bc, T* xc,
                    const CGArgs& g, int conv_it, hipStream_t s);
// the last pair up onto level 0 (2D) with level 0's second post-smoothing and the (b, x)
// partials: x = the V-cycle's result from x2f (read only); false (nothing launched) when
// level 0's tiles are not the partials' blocks
template <class T>
bool launch_mg_up_last(const Grid& G, const Level& c, const T* bc, const T* t1c, const T* t2c, const Level& f,
                       const T* bf, const T* x2f, T* x, const CGArgs& g, hipStream_t s);
template <class T>
void launch_mg_up(const Grid& G, const Level& c, const T* bc, const T* t1c, const T* t2c, const Level& f,
                  const T* bf, const T* x2f, T* t1f, T* t2f, const CGArgs& g, hipStream_t s);

// CG iteration it (1-based): apply (p = z + beta p_old, q = A p, (p,q) partials) and update
// (x += alpha p, r_new = r_old - alpha q, (r,r) partials; with xm != nullptr also the first
// smoothing of the next V-cycle on level 0)
template <class T>
void launch_cg_apply(const Grid& G, const Level& L, const T* z, const T* pold, T* pnew, T* q, T* x,
                     const CGArgs& g, int it, hipStream_t s);
template <class T>
void launch_cg_update(const Grid& G, const Level& L, const T* rold, const T* q, const T* p, T* x, T* rnew,
                      T* xm, const CGArgs& g, int it, hipStream_t s);
// when level 0 is itself the dense coarsest level: control reset with (b,b) partials; the
// convergence decision; the (r,z) partials
template <class T>
void launch_cg_init(int n, const T* b, const CGArgs& g, hipStream_t s);
void launch_cg_decide(const CGArgs& g, int it, hipStream_t s);
template <class T>
void launch_cg_dot_rz(int n, const T* r, const T* z, const CGArgs& g, hipStream_t s);
// double <-> float with scaling by 1/sqrt(*nrm2) (to float) or sqrt(*nrm2) (back)
void launch_cast_scale_f32(size_t n, const double* src, const double* nrm2, float* dst, hipStream_t s);
void launch_uncast_scale_f64(size_t n, const float* src, const double* nrm2, double* dst, hipStream_t s);

// transforms: rhs_p = F_p / (Gamma1 p) (schur: - dt div F_u);  rhs_T = rho F_e + (dp/dt - F_p)/Gamma1;
// z = zscale dX from dp (and dT).  scaled != 0: the input is v with r = L v.  For a
// theta-weighted step dt is the implicit step theta dt and zscale = 1/theta.
void launch_pbp_in(const Grid& G, const double* X, const double* v, int scaled, double alpha1,
                   double dt, int schur, double* rhs_p, hipStream_t s,
                   const double* vn2 = nullptr);
void launch_pbp_rhsT(const Grid& G, const double* X, const double* v, int scaled, double alpha1,
                     double dt, const double* dp, double* rhs_T, hipStream_t s,
                     const double* vn2 = nullptr);
// vn2 (optional, also for pbp_in and pbp_rhsT): v is read as v / sqrt(*vn2), an Arnoldi vector
// kept unnormalised.
// zn2 (optional): *zn2 = ||R^-1 z||_2^2 with the unknown scaling R (alpha2) of X, reduced
// through zn2_ws (the scaled norm of the finite-difference step size, computed with z)
void launch_pbp_out(const Grid& G, const double* X, const double* v, int scaled, double alpha1,
                    double dt, const double* dp, const double* dT, double zscale, double* z, hipStream_t s,
                    double alpha2 = 0.0, const RedWS* zn2_ws = nullptr, double* zn2 = nullptr,
                    const double* vn2 = nullptr);

// ---- transposed products (vjp.hip) -----------------------------------------------------
// out = cU (dU/dX)^T w + cR (dR/dX)^T w at X (optionally each row multiplied by R(X));
// scratch holds vjp_scratch_doubles(G) doubles
size_t vjp_scratch_doubles(const Grid& G);
void launch_vjp(const Grid& G, const double* X, const double* w, double cU, double cR, double* scratch,
                int scaleR, double alpha2, double* out, hipStream_t s);
// transposed preconditioner: rhs of the pressure solve (and of the thermal solve), the
// completion of the pressure rhs after the thermal solve, and the output z = M^-T v
// (scaled != 0: the input is v with w = v / R)
void launch_pbpT_in(const Grid& G, const double* X, const double* v, int scaled, double alpha2,
                    double dt, int thermal, double* rhs_p, double* rhs_T, hipStream_t s);
void launch_pbpT_mid(const Grid& G, const double* X, double dt, const double* t, double* rhs_p, hipStream_t s);
void launch_pbpT_out(const Grid& G, const double* X, const double* v, int scaled, double alpha2,
                     double dt, const double* sp, const double* t, int schur, double zscale, double* z,
                     hipStream_t s);

}  // namespace jfnk
