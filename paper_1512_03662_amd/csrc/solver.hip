// Host side of the implicit-step library: context and workspace, the Newton loop
// (Sect. 4.1), flexible GMRES(m) with CGS2 (Sects. 4.1, 4.3), the physics-based
// preconditioner (Sect. 4.3) and its multigrid-preconditioned CG solves (Sect. 3.5), and
// the C ABI of include/jfnk.h.
//
// Control stays on the host; the device is asked only for scalars (norms, Hessenberg
// columns, CG residuals), so every vector operation runs in the kernels of this library.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/jfnk.h"
#include "kernels.hpp"
#include "probe.hpp"

using namespace jfnk;

namespace {

// device scalar slots
enum Slot {
  S_XN2 = 0,   // ||R^-1 X||^2   (followed by S_ZN2: the finite-difference kernel reads both)
  S_ZN2 = 1,   // ||R^-1 Z_j||^2
  S_FN2 = 2,   // ||L^-1 F||^2
  S_DXMAX = 3, // ||R^-1 dX||_inf   (followed by S_ADM: max -min(rho, e) of the corrected state)
  S_ADM = 4,
  S_TMP = 9,   // ||b||^2 of an FP32 elliptic solve
  S_H1 = 16,                       // h of the first Gram-Schmidt pass (kMaxK)
  S_H2 = S_H1 + kMaxK,             // h of the second pass (kMaxK) then ||w||^2
  S_NRM3 = S_H2 + kMaxK + 1,       // ||w||^2 after the second pass
  S_Y = S_NRM3 + 1,                // least-squares coefficients y (kMaxK)
  S_COUNT = S_Y + kMaxK
};

// coarsest levels with more cells than this are smoothed, not solved by a dense inverse
constexpr int kDenseMaxN = 4096;

struct EllOp {
  std::vector<Level> lv64, lv32;
  double* Ainv = nullptr;   // dense inverse of the coarsest level (null: smoothed bottom)
  int Nc = 0;
  std::vector<double> hA;   // host scratch
};

}  // namespace

struct jfnk_ctx {
  jfnk_problem prob{};
  jfnk_opts opts{};
  Grid G{};
  hipStream_t stream = nullptr;
  int nvar = 0;
  size_t n = 0;          // nvar * N
  int m_alloc = 0;
  double dt = 0.0;
  bool have_state = false;
  std::string err;
  size_t bytes = 0;
  std::vector<void*> allocs;

  // state-sized buffers
  double *bn = nullptr, *Xn = nullptr, *G0 = nullptr, *W = nullptr, *W2 = nullptr,
         *dX = nullptr, *Xk = nullptr /* X + delta Z of the FD product */, *V = nullptr, *Z = nullptr;
  double* scal = nullptr;   // device scalars
  double* hscal = nullptr;  // pinned host mirror
  RedWS red;

  // preconditioner
  EllOp ops[2];
  double *rhs_p = nullptr, *dp = nullptr, *rhs_T = nullptr, *dT = nullptr;
  double* cg64[7] = {};    // r1 r2 p1 p2 q z x2
  float* cg32[9] = {};     // r1 r2 p1 p2 q z x2 b x
  CGCtl* ctl = nullptr;    // control block of the running CG solve
  CGCtl* hctl = nullptr;   // pinned host copy
  double* cgpart = nullptr;
  const double* zn2_of = nullptr;  // the direction whose ||R^-1 z||^2 the preconditioner left in S_ZN2
  int cg_pred[2][2] = {{4, 4}, {4, 4}};  // previous iteration count per operator and precision
  int cg_its = 0;

  // zero "coarse correction" (one element, strides 0) for the smoothing of a bottom level
  double* zero64 = nullptr;
  float* zero32 = nullptr;

  // adjoint
  double* vjps = nullptr;   // scratch of the transposed products
  bool adj = false;         // FGMRES works on the transposed system

  // per-phase GPU time of a step (opts.phase_timing): start/stop event pairs recorded on the
  // stream around each phase, read back after the next host synchronisation
  static constexpr int kPhasePairs = 16;
  hipEvent_t pev[2 * kPhasePairs] = {};
  int pphase[kPhasePairs] = {};
  int pused = 0;
  bool pstarted = false;    // a start event is recorded in slot pused
  double pms[4] = {};       // residual, J.v, preconditioner, orthogonalisation (ms)
};

static std::string g_create_err;

#define HIPX(expr)                                                                     \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      throw DevErr(std::string(#expr) + ": " + hipGetErrorString(e_));               \
    }                                                                                  \
  } while (0)

namespace {

struct DevErr {
  std::string msg;
  explicit DevErr(std::string m) : msg(std::move(m)) {}
};
struct InvErr {
  std::string msg;
  explicit InvErr(std::string m) : msg(std::move(m)) {}
};
struct FiniteErr {
  std::string msg;
  explicit FiniteErr(std::string m) : msg(std::move(m)) {}
};
struct AdmissErr {
  std::string msg;
  explicit AdmissErr(std::string m) : msg(std::move(m)) {}
};

template <class T>
T* dalloc(jfnk_ctx* c, size_t count) {
  void* p = nullptr;
  size_t b = std::max<size_t>(count, 1) * sizeof(T);
  HIPX(hipMalloc(&p, b));
  c->allocs.push_back(p);
  c->bytes += b;
  return (T*)p;
}

void check_launch() { HIPX(hipGetLastError()); }

void sync(jfnk_ctx* c) { HIPX(hipStreamSynchronize(c->stream)); }

// copy device scalars [first, first+count) to the host mirror and wait
// ---- per-phase timing ----------------------------------------------------------------------
enum Phase { PH_RESID = 0, PH_JV = 1, PH_PREC = 2, PH_ORTH = 3 };

// adds the elapsed times of the recorded pairs (the stream has been synchronised)
void phase_flush(jfnk_ctx* c) {
  for (int i = 0; i < c->pused; ++i) {
    float ms = 0.0f;
    HIPX(hipEventElapsedTime(&ms, c->pev[2 * i], c->pev[2 * i + 1]));
    c->pms[c->pphase[i]] += ms;
  }
  c->pused = 0;
}

void phase_begin(jfnk_ctx* c) {
  if (!c->opts.phase_timing) return;
  if (!c->pev[0])
    for (auto& e : c->pev) HIPX(hipEventCreate(&e));
  if (c->pused == jfnk_ctx::kPhasePairs) {  // pool full: wait for the recorded pairs
    HIPX(hipStreamSynchronize(c->stream));
    phase_flush(c);
  }
  HIPX(hipEventRecord(c->pev[2 * c->pused], c->stream));
  c->pstarted = true;
}

void phase_end(jfnk_ctx* c, int ph) {
  if (!c->opts.phase_timing || !c->pstarted) return;
  HIPX(hipEventRecord(c->pev[2 * c->pused + 1], c->stream));
  c->pphase[c->pused++] = ph;
  c->pstarted = false;
}

void pull(jfnk_ctx* c, int first, int count) {
  check_launch();
  HIPX(hipMemcpyAsync(c->hscal + first, c->scal + first, count * sizeof(double),
                      hipMemcpyDeviceToHost, c->stream));
  sync(c);
  if (c->pused) phase_flush(c);
}

// starts a step's phase clocks; phase_finish writes them into the step's statistics
void phase_start(jfnk_ctx* c) {
  c->pused = 0;
  c->pstarted = false;
  for (double& v : c->pms) v = 0.0;
}
void phase_finish(jfnk_ctx* c, jfnk_step_stats* S) {
  if (c->opts.phase_timing) {
    sync(c);
    phase_flush(c);
  }
  S->t_resid = c->pms[PH_RESID];
  S->t_jv = c->pms[PH_JV];
  S->t_prec = c->pms[PH_PREC];
  S->t_orth = c->pms[PH_ORTH];
}

void push(jfnk_ctx* c, int first, int count) {
  HIPX(hipMemcpyAsync(c->scal + first, c->hscal + first, count * sizeof(double),
                      hipMemcpyHostToDevice, c->stream));
}

void copy_d2d(jfnk_ctx* c, void* dst, const void* src, size_t bytes) {
  HIPX(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream));
}

Grid make_grid(const jfnk_problem& p) {
  Grid G{};
  G.nd = p.ndim;
  for (int d = 0; d < 3; ++d) {
    G.n[d] = (d < p.ndim) ? p.n[d] : 1;
    G.bc[d] = (d < p.ndim) ? p.bc[d] : 0;
    G.dx[d] = (d < p.ndim) ? p.dx[d] : 1.0;
    G.idx[d] = 1.0 / G.dx[d];
    G.g[d] = (d < p.ndim) ? p.g[d] : 0.0;
    G.qwall[d][0] = p.qwall[d][0];
    G.qwall[d][1] = p.qwall[d][1];
  }
  G.stride[0] = 1;
  G.stride[1] = G.n[0];
  G.stride[2] = G.n[0] * G.n[1];
  G.N = G.n[0] * G.n[1] * G.n[2];
  G.gamma = p.gamma;
  G.chi_model = p.chi_model;
  G.chi0 = p.chi0;
  G.chi_tref_inv = 1.0 / p.chi_tref;
  G.chi_exp = p.chi_exp;
  G.theta = p.theta;
  G.a_rad = p.a_rad;
  return G;
}

void validate_problem(const jfnk_problem* p) {
  if (!p) throw InvErr("null problem");
  if (p->ndim != 2 && p->ndim != 3) throw InvErr("ndim must be 2 or 3");
  double cells = 1.0;
  for (int d = 0; d < p->ndim; ++d) {
    if (p->n[d] < 4) throw InvErr("every axis needs at least 4 cells");
    if (!(p->dx[d] > 0.0)) throw InvErr("dx must be positive");
    if (p->bc[d] != JFNK_BC_PERIODIC && p->bc[d] != JFNK_BC_WALL) throw InvErr("bad bc");
    cells *= p->n[d];
  }
  if (p->ndim == 2 && p->n[2] != 1) throw InvErr("n[2] must be 1 in 2D");
  if (cells * (2 + p->ndim) > 2.0e9) throw InvErr("grid too large for 32-bit cell indexing");
  if (!(p->gamma > 1.0)) throw InvErr("gamma must exceed 1");
  if (p->chi_model < 0 || p->chi_model > 2) throw InvErr("bad chi_model");
  if (p->chi_model != JFNK_CHI_NONE && !(p->chi0 >= 0.0)) throw InvErr("chi0 must be >= 0");
  if (p->chi_model == JFNK_CHI_POWER && !(p->chi_tref > 0.0)) throw InvErr("chi_tref must be > 0");
  if (!(p->theta > 0.0 && p->theta <= 1.0)) throw InvErr("theta must be in (0, 1]");
  if (!(p->a_rad >= 0.0 && p->a_rad < HUGE_VAL)) throw InvErr("a_rad must be finite and >= 0");
}

void validate(const jfnk_problem* p, const jfnk_opts* o) {
  if (!p || !o) throw InvErr("null problem or options");
  validate_problem(p);
  if (o->gmres_m < 1 || o->gmres_m > kMaxK - 2) throw InvErr("gmres_m out of range");
  if (o->gmres_maxit < 1) throw InvErr("gmres_maxit must be >= 1");
  if (o->newton_max < 1 || o->newton_min < 1) throw InvErr("newton_max/newton_min must be >= 1");
  if (o->jv_mode != JFNK_JV_FD && o->jv_mode != JFNK_JV_EXACT) throw InvErr("bad jv_mode");
  if (o->precond < 0 || o->precond > 2) throw InvErr("bad precond");
  if (o->ell_precision != JFNK_FP64 && o->ell_precision != JFNK_FP32) throw InvErr("bad ell_precision");
  if (o->cg_maxit < 0) throw InvErr("cg_maxit must be >= 0");
  if (o->pc_schur != 0 && o->pc_schur != 1) throw InvErr("pc_schur must be 0 or 1");
  if (o->phase_timing != 0 && o->phase_timing != 1) throw InvErr("phase_timing must be 0 or 1");
  if (o->mg_levels < 0) throw InvErr("mg_levels must be >= 0");
  if (o->mg_smooth < 0 || o->mg_smooth > 8) throw InvErr("mg_smooth (Chebyshev degree) must be in 1..8 (0: 2)");
}

}  // namespace

namespace jfnk {
// Grid of a problem; a non-empty return is the reason the problem is refused.
std::string grid_of_problem(const jfnk_problem* p, Grid* G) {
  try {
    validate_problem(p);
    *G = make_grid(*p);
  } catch (const InvErr& e) {
    return e.msg;
  }
  return std::string();
}
// message returned by jfnk_last_error(NULL) for calls made without a context
void set_context_free_error(const std::string& msg) { g_create_err = msg; }
}  // namespace jfnk

namespace {

// ---- multigrid hierarchy ----------------------------------------------------------------
bool coarsenable(const int* n, int nd) {
  for (int d = 0; d < nd; ++d)
    if (n[d] % 2 != 0 || n[d] <= 4) return false;
  return true;
}

Level make_level(jfnk_ctx* c, const int* n, int nd, bool f32, bool level0) {
  Level L;
  for (int d = 0; d < 3; ++d) L.n[d] = (d < nd) ? n[d] : 1;
  L.stride[0] = 1;
  L.stride[1] = L.n[0];
  L.stride[2] = L.n[0] * L.n[1];
  L.N = L.n[0] * L.n[1] * L.n[2];
  size_t es = f32 ? sizeof(float) : sizeof(double);
  auto al = [&](void) -> void* {
    void* p = nullptr;
    HIPX(hipMalloc(&p, std::max<size_t>(L.N, 1) * es));
    c->allocs.push_back(p);
    c->bytes += L.N * es;
    return p;
  };
  L.diag = al();
  for (int d = 0; d < nd; ++d) L.w[d] = al();
  L.dinv = al();
  if (!level0) {
    L.b = al();
    L.x = al();
  }
  L.t1 = al();
  L.t2 = al();
  return L;
}

void build_hierarchy(jfnk_ctx* c, EllOp& op, bool want32) {
  const Grid& G = c->G;
  int n[3] = {G.n[0], G.n[1], G.n[2]};
  op.lv64.push_back(make_level(c, n, G.nd, false, true));
  if (want32) op.lv32.push_back(make_level(c, n, G.nd, true, true));
  const int maxl = c->opts.mg_levels;  // 0: as deep as the grid allows
  while (coarsenable(n, G.nd) && (maxl == 0 || (int)op.lv64.size() < maxl)) {
    for (int d = 0; d < G.nd; ++d) n[d] /= 2;
    op.lv64.push_back(make_level(c, n, G.nd, false, false));
    if (want32) op.lv32.push_back(make_level(c, n, G.nd, true, false));
  }
  op.Nc = op.lv64.back().N;
  // an odd axis stops the coarsening; a coarsest level too large for the dense inverse is
  // smoothed instead (see bottom_smooth)
  if (op.Nc <= kDenseMaxN) {
    op.Ainv = dalloc<double>(c, (size_t)op.Nc * op.Nc);
    op.hA.resize((size_t)op.Nc * op.Nc);
  }
}

// dense inverse of the SPD coarsest operator (Cholesky), built on the host from the
// level's coefficients
void coarse_setup(jfnk_ctx* c, EllOp& op) {
  const Grid& G = c->G;
  const Level& L = op.lv64.back();
  int N = L.N;
  std::vector<double> diag(N), w[3];
  HIPX(hipMemcpyAsync(diag.data(), L.diag, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  for (int d = 0; d < G.nd; ++d) {
    w[d].resize(N);
    HIPX(hipMemcpyAsync(w[d].data(), L.w[d], N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  }
  sync(c);
  std::vector<double>& A = op.hA;
  std::fill(A.begin(), A.end(), 0.0);
  for (int lin = 0; lin < N; ++lin) {
    A[(size_t)lin * N + lin] += diag[lin];
    int cc[3] = {lin % L.n[0], (lin / L.n[0]) % L.n[1], lin / (L.n[0] * L.n[1])};
    for (int d = 0; d < G.nd; ++d) {
      int nd_ = L.n[d];
      int m = (cc[d] == 0) ? lin + (nd_ - 1) * L.stride[d] : lin - L.stride[d];
      double wf = w[d][lin];
      A[(size_t)lin * N + lin] += wf;
      A[(size_t)m * N + m] += wf;
      A[(size_t)lin * N + m] -= wf;
      A[(size_t)m * N + lin] -= wf;
    }
  }
  // Cholesky A = C C^T (lower), then A^-1 = C^-T C^-1
  std::vector<double> C(A);
  for (int j = 0; j < N; ++j) {
    double s = C[(size_t)j * N + j];
    for (int k = 0; k < j; ++k) s -= C[(size_t)j * N + k] * C[(size_t)j * N + k];
    if (!(s > 0.0)) throw FiniteErr("coarse multigrid operator is not positive definite");
    double djj = std::sqrt(s);
    C[(size_t)j * N + j] = djj;
    for (int i = j + 1; i < N; ++i) {
      double t = C[(size_t)i * N + j];
      for (int k = 0; k < j; ++k) t -= C[(size_t)i * N + k] * C[(size_t)j * N + k];
      C[(size_t)i * N + j] = t / djj;
    }
  }
  // columns of C^-1 by forward substitution, then A^-1 = C^-T C^-1
  std::vector<double> Ci((size_t)N * N, 0.0);
  for (int col = 0; col < N; ++col) {
    for (int i = 0; i < N; ++i) {
      double t = (i == col) ? 1.0 : 0.0;
      for (int k = col; k < i; ++k) t -= C[(size_t)i * N + k] * Ci[(size_t)k * N + col];
      Ci[(size_t)i * N + col] = (i < col) ? 0.0 : t / C[(size_t)i * N + i];
    }
  }
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double s = 0.0;
      for (int k = std::max(i, j); k < N; ++k) s += Ci[(size_t)k * N + i] * Ci[(size_t)k * N + j];
      A[(size_t)i * N + j] = s;
    }
  HIPX(hipMemcpyAsync(op.Ainv, A.data(), (size_t)N * N * sizeof(double), hipMemcpyHostToDevice,
                      c->stream));
  sync(c);  // the host buffer is reused
}

void ell_setup(jfnk_ctx* c, const double* X, double dt) {
  const Grid& G = c->G;
  int nops = (c->opts.precond == JFNK_PC_SOUND_THERMAL) ? 2 : 1;
  for (int o = 0; o < nops; ++o) {
    EllOp& op = c->ops[o];
    Level& L0 = op.lv64[0];
    double* w[3] = {(double*)L0.w[0], (double*)L0.w[1], (double*)L0.w[2]};
    launch_ell_coef(G, X, dt, o, (double*)L0.diag, w, c->stream);
    for (size_t l = 0; l + 1 < op.lv64.size(); ++l)
      launch_ell_coarsen<double>(G, op.lv64[l], op.lv64[l + 1], c->stream);
    for (auto& L : op.lv64) launch_ell_dinv<double>(G, L, c->stream);
    if (c->opts.ell_precision == JFNK_FP32)
      for (size_t l = 0; l < op.lv64.size(); ++l) launch_level_to_f32(op.lv64[l], op.lv32[l], G.nd, c->stream);
    check_launch();
    if (op.Ainv) coarse_setup(c, op);
  }
}

// The bottom of a V-cycle on level L: x = A^-1 b by the dense inverse, or, when the level is
// too large for it, the degree-2 Chebyshev smoothing from zero (into xs) followed by the same
// smoothing from that iterate (a "prolongation" of a zero coarse vector, then the second
// smoothing), which keeps the V-cycle symmetric positive definite.
template <class T>
void bottom_solve(jfnk_ctx* c, const Level& L, const double* Ainv, const T* b, T* xs, T* x, const CGArgs& g) {
  const Grid& G = c->G;
  hipStream_t s = c->stream;
  if (Ainv) {
    launch_dense_matvec<T>(L.N, Ainv, b, x, g, s);
    return;
  }
  Level zc{};
  zc.N = 1;  // strides 0: every cell's parent is the single zero entry
  const T* zero = std::is_same<T, float>::value ? (const T*)c->zero32 : (const T*)c->zero64;
  launch_mg_presmooth<T>(G, L, b, xs, g, false, s);
  launch_mg_prolong_smooth1<T>(G, L, b, xs, zero, zc, (T*)L.t1, (T*)L.t2, g, s);
  launch_mg_smooth2<T>(G, L, b, (const T*)L.t1, (const T*)L.t2, x, g, false, s);
}

// first level handled by the single-workgroup coarse kernel (nl - 1 when the coarsest
// level is too large for it and is solved by the dense inverse alone)
int first_fused(const std::vector<Level>& lv, bool* fused) {
  const int nl = (int)lv.size();
  int l0 = nl - 1;
  *fused = lv[nl - 1].N <= kCoarseMaxN;
  if (*fused)
    while (l0 > 0 && lv[l0 - 1].N <= kCoarseMaxN && nl - (l0 - 1) <= kMaxLevels) --l0;
  return l0;
}

// The V-cycle z = M r after level 0's first smoothing (in x2, read only), ending with the
// (r, z) partials; with it > 0 the convergence decision of iteration it is taken on the way
// down.  Requires first_fused(lv) >= 1.  When the coarsest levels run in the single-workgroup
// kernel, level pairs are fused: down(l -> l+1) = restriction + first smoothing of l+1,
// up(l -> l-1) = second smoothing of l + prolongation and first post-smoothing of l-1; the
// coarse kernel starts from the first smoothing of its first level and stops after that
// level's first post-smoothing step.  On 2D grids the last pair up also takes level 0's
// second post-smoothing when its tiles are the partials' blocks.
template <class T>
void vcycle_rest(jfnk_ctx* c, std::vector<Level>& lv, const double* Ainv, const T* r, T* x2, T* z,
                 const CGArgs& g, int it) {
  const Grid& G = c->G;
  hipStream_t s = c->stream;
  const int nl = (int)lv.size();
  bool fused;
  const int l0 = first_fused(lv, &fused);
  auto B = [&](int l) -> const T* { return l == 0 ? r : (const T*)lv[l].b; };
  // the level's iterate as read on the way down and into the prolongation (x2 on level 0)
  auto Xl = [&](int l) -> T* { return l == 0 ? x2 : (T*)lv[l].x; };
  if (fused) {
    // a pair is fused while its coarse level is small (launch-latency bound); on large levels
    // the halo recomputation costs more than the launch it saves
    auto fuse = [&](int lc) { return lv[lc].N <= kFusePairMaxN; };
    // when the fused part is the coarsest level alone it is solved exactly, without smoothing:
    // the last pair down is a plain restriction and the first pair up a plain prolongation
    const bool single = (nl - l0 == 1);
    const int ltop = single ? l0 - 1 : l0;
    for (int l = 0; l < ltop; ++l) {
      const int conv = (l == 0) ? it : 0;
      if (fuse(l + 1)) {
        launch_mg_down<T>(G, lv[l], B(l), Xl(l), lv[l + 1], (T*)lv[l + 1].b, (T*)lv[l + 1].x, g, conv, s);
      } else {
        launch_mg_restrict_resid<T>(G, lv[l], B(l), Xl(l), (T*)lv[l + 1].b, lv[l + 1], g, conv, s);
        launch_mg_presmooth<T>(G, lv[l + 1], B(l + 1), Xl(l + 1), g, false, s);
      }
    }
    if (single) {
      const int lp = l0 - 1;
      launch_mg_restrict_resid<T>(G, lv[lp], B(lp), Xl(lp), (T*)lv[l0].b, lv[l0], g, lp == 0 ? it : 0, s);
      launch_vcycle_coarse<T>(G, &lv[l0], 1, Ainv, B(l0), Xl(l0), g, 0, 0, s);
      launch_mg_prolong_smooth1<T>(G, lv[lp], B(lp), Xl(lp), Xl(l0), lv[l0], (T*)lv[lp].t1, (T*)lv[lp].t2, g, s);
    } else {
      launch_vcycle_coarse<T>(G, &lv[l0], nl - l0, Ainv, B(l0), Xl(l0), g, kCoarseFromPre | kCoarseToUp, 0, s);
    }
    for (int l = ltop; l >= 1; --l) {
      if (fuse(l)) {
        if (l == 1 && launch_mg_up_last<T>(G, lv[1], B(1), (const T*)lv[1].t1, (const T*)lv[1].t2, lv[0], r, x2,
                                           z, g, s))
          return;
        launch_mg_up<T>(G, lv[l], B(l), (const T*)lv[l].t1, (const T*)lv[l].t2, lv[l - 1], B(l - 1), Xl(l - 1),
                        (T*)lv[l - 1].t1, (T*)lv[l - 1].t2, g, s);
      } else {
        launch_mg_smooth2<T>(G, lv[l], B(l), (const T*)lv[l].t1, (const T*)lv[l].t2, Xl(l), g, false, s);
        launch_mg_prolong_smooth1<T>(G, lv[l - 1], B(l - 1), Xl(l - 1), Xl(l), lv[l], (T*)lv[l - 1].t1,
                                     (T*)lv[l - 1].t2, g, s);
      }
    }
    launch_mg_smooth2<T>(G, lv[0], r, (const T*)lv[0].t1, (const T*)lv[0].t2, z, g, true, s);
    return;
  }
  // coarsest level solved by its dense inverse alone: one kernel per V-cycle piece
  launch_mg_restrict_resid<T>(G, lv[0], r, x2, (T*)lv[1].b, lv[1], g, it, s);
  for (int l = 1; l < l0; ++l) {
    launch_mg_presmooth<T>(G, lv[l], B(l), Xl(l), g, false, s);
    launch_mg_restrict_resid<T>(G, lv[l], B(l), Xl(l), (T*)lv[l + 1].b, lv[l + 1], g, 0, s);
  }
  bottom_solve<T>(c, lv[nl - 1], Ainv, B(nl - 1), Xl(nl - 1), Xl(nl - 1), g);
  for (int l = l0 - 1; l >= 0; --l) {
    launch_mg_prolong_smooth1<T>(G, lv[l], B(l), Xl(l), Xl(l + 1), lv[l + 1], (T*)lv[l].t1,
                                 (T*)lv[l].t2, g, s);
    launch_mg_smooth2<T>(G, lv[l], B(l), (const T*)lv[l].t1, (const T*)lv[l].t2, l == 0 ? z : Xl(l), g, l == 0,
                         s);
  }
}

// One V-cycle z = M r with the Chebyshev smoother of degree k != 2 (opts.mg_smooth), one
// launch per smoothing step on every level (the fused kernels above implement degree 2).  On
// level l the result goes to out (lv[l].x, or z on level 0); the presmoothed iterate is kept
// in `pre` for the restriction and the prolongation, and the smoother's x iterates alternate
// so that the last step of each smoothing lands where it must (steps never read and write
// the same x buffer; d is updated in place).  The coarsest level is solved by its dense
// inverse, or, above the dense limit, smoothed from zero and then from that iterate.
template <class T>
void vcycle_any(jfnk_ctx* c, std::vector<Level>& lv, const double* Ainv, int l, const T* b, T* out, T* other, T* d,
                const CGArgs& g, int k) {
  const Grid& G = c->G;
  hipStream_t s = c->stream;
  const int nl = (int)lv.size();
  double c1[16], c2[16];
  cheb_coefs(k, c1, c2);
  // the presmoothed iterate sits in `out` when k is even and in `other` when k is odd, so that
  // the post-smoothing (which starts by reading it and alternates from the other buffer)
  // ends in `out`
  T* pre = (k % 2 == 0) ? out : other;
  T* alt = (k % 2 == 0) ? other : out;
  // k steps from zero, ending in pre
  auto smooth_zero = [&]() {
    T* y = ((k - 1) % 2 == 0) ? pre : alt;
    launch_cheb_zero<T>(G, lv[l], b, y, d, g, s);
    for (int i = 1; i < k; ++i) {
      T* yn = ((k - 1 - i) % 2 == 0) ? pre : alt;
      launch_cheb_step<T>(G, lv[l], b, y, yn, d, c1[i], c2[i], g, s);
      y = yn;
    }
  };
  // k steps from pre + P xc (xc on level C), ending in out
  auto smooth_post = [&](const T* xc, const Level& C) {
    launch_mg_prolong_smooth1<T>(G, lv[l], b, pre, xc, C, alt, d, g, s);
    T* y = alt;
    for (int i = 1; i < k; ++i) {
      T* yn = (y == alt) ? pre : alt;
      launch_cheb_step<T>(G, lv[l], b, y, yn, d, c1[i], c2[i], g, s);
      y = yn;
    }
  };
  if (l == nl - 1) {
    if (Ainv) {
      launch_dense_matvec<T>(lv[l].N, Ainv, b, out, g, s);
      return;
    }
    Level zc{};
    zc.N = 1;  // strides 0: every cell's parent is the single zero entry
    const T* zero = std::is_same<T, float>::value ? (const T*)c->zero32 : (const T*)c->zero64;
    smooth_zero();
    smooth_post(zero, zc);
    return;
  }
  smooth_zero();
  Level& C = lv[l + 1];
  launch_mg_restrict_resid<T>(G, lv[l], b, pre, (T*)C.b, C, g, 0, s);
  vcycle_any<T>(c, lv, Ainv, l + 1, (const T*)C.b, (T*)C.x, (T*)C.t1, (T*)C.t2, g, k);
  smooth_post((const T*)C.x, C);
}

// PCG as below with the V-cycle of vcycle_any (smoother degree k != 2): the decision of each
// iteration is a kernel of its own, and the (r, z) partials a dot product after the V-cycle.
template <class T>
int pcg_any(jfnk_ctx* c, std::vector<Level>& lv, const double* Ainv, const T* b, T* x, T* const* v, int* pred,
            const CGArgs& g, int k) {
  const Grid& G = c->G;
  hipStream_t s = c->stream;
  const int N = G.N;
  T *r1 = v[0], *r2 = v[1], *p1 = v[2], *p2 = v[3], *q = v[4], *z = v[5], *x2 = v[6];
  T* d = (T*)lv[0].t2;
  launch_cg_init<T>(N, b, g, s);
  if (g.maxit == 0) {
    vcycle_any<T>(c, lv, Ainv, 0, b, x, x2, d, g, k);
    return 0;
  }
  vcycle_any<T>(c, lv, Ainv, 0, b, z, x2, d, g, k);
  launch_cg_dot_rz<T>(N, b, z, g, s);
  const T* rold = b;
  T* rnew = r1;
  const T* pold = z;
  T* pnew = p1;
  int enq = 0;
  int batch = std::max(1, std::min(*pred, g.maxit));
  for (;;) {
    for (int i = 0; i < batch && enq < g.maxit; ++i) {
      const int it = ++enq;
      const bool last = (enq == g.maxit) || (i == batch - 1);
      launch_cg_apply<T>(G, lv[0], z, pold, pnew, q, x, g, it, s);
      launch_cg_update<T>(G, lv[0], rold, q, pnew, x, rnew, nullptr, g, it, s);
      launch_cg_decide(g, it, s);
      if (!last) {
        vcycle_any<T>(c, lv, Ainv, 0, rnew, z, x2, d, g, k);
        launch_cg_dot_rz<T>(N, rnew, z, g, s);
      }
      rold = rnew;
      rnew = (rnew == r1) ? r2 : r1;
      pold = pnew;
      pnew = (pnew == p1) ? p2 : p1;
    }
    check_launch();
    HIPX(hipMemcpyAsync(c->hctl, c->ctl, sizeof(CGCtl), hipMemcpyDeviceToHost, s));
    sync(c);
    if (c->hctl->flag != 0 || enq >= g.maxit) break;
    vcycle_any<T>(c, lv, Ainv, 0, rold, z, x2, d, g, k);
    launch_cg_dot_rz<T>(N, rold, z, g, s);
    batch = 1;
  }
  if (c->hctl->flag < 0) throw FiniteErr("non-finite residual in an elliptic solve");
  if (c->hctl->flag == 0) throw FiniteErr("elliptic solve ended without a decision");
  *pred = std::max(1, c->hctl->its);
  return c->hctl->its;
}

// PCG on level 0 of lv: x = A^-1 b (x and b of type T, length N), stopping when
// ||r|| < cg_eta ||b|| or after cg_maxit iterations.  The iterations run from the device
// (CGCtl); the host enqueues `pred` of them (the previous count of this solver), then one
// at a time until the control block reports a stop.  v: r1, r2, p1, p2, q, z, x2 (x2: level 0's
// iterate after its first smoothing, the V-cycle's input; z its output).
template <class T>
int pcg(jfnk_ctx* c, std::vector<Level>& lv, const double* Ainv, const T* b, T* x, T* const* v,
        int* pred) {
  const Grid& G = c->G;
  hipStream_t s = c->stream;
  const int N = G.N;
  T *r1 = v[0], *r2 = v[1], *p1 = v[2], *p2 = v[3], *q = v[4], *z = v[5], *x2 = v[6];
  CGArgs g;
  g.ctl = c->ctl;
  g.part = c->cgpart;
  g.np = cg_partials((size_t)N);
  g.eta = c->opts.cg_eta;
  g.maxit = c->opts.cg_maxit;
  const int deg = (c->opts.mg_smooth == 0) ? 2 : c->opts.mg_smooth;
  if (deg != 2) return pcg_any<T>(c, lv, Ainv, b, x, v, pred, g, deg);
  bool fused;
  const int l0 = first_fused(lv, &fused);
  const int nl = (int)lv.size();
  // cg_maxit = 0: the solve is one V-cycle, x = M b (a fixed symmetric linear operator); no
  // CG step and no host synchronisation
  if (g.maxit == 0) z = x;
  // z = M b with the (b, b) and (b, z) partials
  if (l0 >= 1) {
    launch_mg_presmooth<T>(G, lv[0], b, x2, g, true, s);
    vcycle_rest<T>(c, lv, Ainv, b, x2, z, g, 0);
  } else if (fused) {
    launch_vcycle_coarse<T>(G, &lv[0], nl, Ainv, b, z, g, kCoarseInit | kCoarseRZ, 0, s);
  } else {
    launch_cg_init<T>(N, b, g, s);
    bottom_solve<T>(c, lv[0], Ainv, b, x2, z, g);
    launch_cg_dot_rz<T>(N, b, z, g, s);
  }
  if (g.maxit == 0) return 0;
  const T* rold = b;
  T* rnew = r1;
  const T* pold = z;
  T* pnew = p1;
  int enq = 0;
  int batch = std::max(1, std::min(*pred, g.maxit));
  for (;;) {
    for (int k = 0; k < batch && enq < g.maxit; ++k) {
      const int it = ++enq;
      // the last iteration of a batch (or the last allowed one) only takes the decision: the
      // next V-cycle is enqueued after the host has read it, and only if the solve goes on
      const bool last = (enq == g.maxit) || (k == batch - 1);
      launch_cg_apply<T>(G, lv[0], z, pold, pnew, q, x, g, it, s);
      launch_cg_update<T>(G, lv[0], rold, q, pnew, x, rnew, (l0 >= 1 && !last) ? x2 : nullptr, g, it, s);
      if (last) {
        launch_cg_decide(g, it, s);
      } else if (l0 >= 1) {
        vcycle_rest<T>(c, lv, Ainv, rnew, x2, z, g, it);
      } else if (fused) {
        launch_vcycle_coarse<T>(G, &lv[0], nl, Ainv, rnew, z, g, kCoarseConv | kCoarseRZ, it, s);
      } else {
        launch_cg_decide(g, it, s);
        bottom_solve<T>(c, lv[0], Ainv, rnew, x2, z, g);
        launch_cg_dot_rz<T>(N, rnew, z, g, s);
      }
      rold = rnew;
      rnew = (rnew == r1) ? r2 : r1;
      pold = pnew;
      pnew = (pnew == p1) ? p2 : p1;
    }
    check_launch();
    HIPX(hipMemcpyAsync(c->hctl, c->ctl, sizeof(CGCtl), hipMemcpyDeviceToHost, s));
    sync(c);
    if (c->hctl->flag != 0 || enq >= g.maxit) break;
    // the solve goes on: z = M r for the last residual (with the first level-0 smoothing that
    // the update kernel skipped); the repeated decision in the V-cycle finds "go on" again
    if (l0 >= 1) {
      launch_mg_presmooth<T>(G, lv[0], rold, x2, g, false, s);
      vcycle_rest<T>(c, lv, Ainv, rold, x2, z, g, enq);
    } else if (fused) {
      launch_vcycle_coarse<T>(G, &lv[0], nl, Ainv, rold, z, g, kCoarseConv | kCoarseRZ, enq, s);
    } else {
      bottom_solve<T>(c, lv[0], Ainv, rold, x2, z, g);
      launch_cg_dot_rz<T>(N, rold, z, g, s);
    }
    batch = 1;
  }
  if (c->hctl->flag < 0) throw FiniteErr("non-finite residual in an elliptic solve");
  if (c->hctl->flag == 0) throw FiniteErr("elliptic solve ended without a decision");
  *pred = std::max(1, c->hctl->its);
  return c->hctl->its;
}

// x = A_op^-1 b in the configured precision (FP32: b normalised by ||b|| before the cast)
void ell_solve(jfnk_ctx* c, int o, const double* b, double* x) {
  EllOp& op = c->ops[o];
  size_t N = (size_t)c->G.N;
  if (c->opts.ell_precision == JFNK_FP64) {
    c->cg_its += pcg<double>(c, op.lv64, op.Ainv, b, x, c->cg64, &c->cg_pred[o][0]);
  } else {
    launch_dot<double>(N, b, b, c->scal + S_TMP, c->red, c->stream);
    float* b32 = c->cg32[7];
    float* x32 = c->cg32[8];
    // S_TMP keeps ||b||^2 for the way back (a zero b gives b32 = 0 and x = 0)
    launch_cast_scale_f32(N, b, c->scal + S_TMP, b32, c->stream);
    c->cg_its += pcg<float>(c, op.lv32, op.Ainv, b32, x32, c->cg32, &c->cg_pred[o][1]);
    launch_uncast_scale_f64(N, x32, c->scal + S_TMP, x, c->stream);
  }
}

// Implicit time step of the semi-implicit scheme: a theta-weighted step has
// J = dU/dX / dt - theta dR/dX = theta (dU/dX / tau - dR/dX) with tau = theta dt, so the
// scheme is built with tau and its result divided by theta (eq. crank_nicholson).
double si_dt(const jfnk_ctx* c) { return c->prob.theta * c->dt; }

// Z = M^-1 v (scaled = 1: v is a scaled basis vector, r = L v) at the frozen state X;
// with_norm: also ||R^-1 Z||^2 into S_ZN2 (the finite-difference product's step size)
// vn2: v is an Arnoldi vector kept unnormalised, read as v / sqrt(*vn2)
void precond(jfnk_ctx* c, const double* X, const double* v, int scaled, double* z, bool with_norm = false,
             const double* vn2 = nullptr) {
  const Grid& G = c->G;
  hipStream_t s = c->stream;
  const jfnk_opts& o = c->opts;
  if (o.precond == JFNK_PC_NONE) {
    if (scaled) launch_scale_LR(G, X, o.alpha2, 1, v, z, 1, s);
    else copy_d2d(c, z, v, c->n * sizeof(double));
    return;
  }
  const double tau = si_dt(c);
  launch_pbp_in(G, X, v, scaled, o.alpha1, tau, o.pc_schur, c->rhs_p, s, vn2);
  ell_solve(c, 0, c->rhs_p, c->dp);
  const double* dT = nullptr;
  if (o.precond == JFNK_PC_SOUND_THERMAL) {
    launch_pbp_rhsT(G, X, v, scaled, o.alpha1, tau, c->dp, c->rhs_T, s, vn2);
    ell_solve(c, 1, c->rhs_T, c->dT);
    dT = c->dT;
  }
  launch_pbp_out(G, X, v, scaled, o.alpha1, tau, c->dp, dT, 1.0 / c->prob.theta, z, s, o.alpha2,
                 with_norm ? &c->red : nullptr, with_norm ? c->scal + S_ZN2 : nullptr, vn2);
  c->zn2_of = with_norm ? z : nullptr;
  check_launch();
}

// Z = M^-T v (scaled = 1: v is a scaled basis vector of the transposed system, w = R^-1 v)
void precond_T(jfnk_ctx* c, const double* X, const double* v, int scaled, double* z) {
  const Grid& G = c->G;
  hipStream_t s = c->stream;
  const jfnk_opts& o = c->opts;
  if (o.precond == JFNK_PC_NONE) {
    if (scaled) launch_scale_LR(G, X, o.alpha1, 0, v, z, 0, s);
    else copy_d2d(c, z, v, c->n * sizeof(double));
    return;
  }
  const bool thermal = (o.precond == JFNK_PC_SOUND_THERMAL);
  const double tau = si_dt(c);
  launch_pbpT_in(G, X, v, scaled, o.alpha2, tau, thermal ? 1 : 0, c->rhs_p, c->rhs_T, s);
  const double* t = nullptr;
  if (thermal) {
    ell_solve(c, 1, c->rhs_T, c->dT);
    launch_pbpT_mid(G, X, tau, c->dT, c->rhs_p, s);
    t = c->dT;
  }
  ell_solve(c, 0, c->rhs_p, c->dp);
  launch_pbpT_out(G, X, v, scaled, o.alpha2, tau, c->dp, t, o.pc_schur, 1.0 / c->prob.theta, z, s);
  check_launch();
}

// out = L^-1 J z at X (scaled operator of eq. jacobian_system_norm applied to an unscaled z)
void apply_J(jfnk_ctx* c, const double* X, const double* z, double* out) {
  const Grid& G = c->G;
  if (c->adj) {
    // transposed system: out = R J^T z
    launch_vjp(G, X, z, 1.0 / c->dt, -c->prob.theta, c->vjps, 1, c->opts.alpha2, out, c->stream);
    return;
  }
  ResidArgs a;
  a.X = X;
  a.V = z;
  a.out = out;
  a.cU = 1.0 / c->dt;
  a.cR = -c->prob.theta;
  a.scaleL = 1;
  a.alpha1 = c->opts.alpha1;
  if (c->opts.jv_mode == JFNK_JV_EXACT) {
    launch_resid(G, a, 1, c->stream);
  } else {
    if (c->zn2_of != z) launch_scaled_norm2(G, X, z, c->opts.alpha2, c->scal + S_ZN2, c->red, c->stream);
    c->zn2_of = nullptr;
    a.B = c->G0;
    a.fd_norms = c->scal + S_XN2;
    a.fd_lambda = c->opts.fd_lambda;
    a.shift = c->Xk;
    launch_resid(G, a, 2, c->stream);
  }
}

// plane rotation (c, s) that zeroes b in (a, b)
void givens(double a, double b, double* c, double* s) {
  if (b == 0.0) {
    *c = 1.0;
    *s = 0.0;
  } else {
    const double r = std::hypot(a, b);
    *c = a / r;
    *s = b / r;
  }
}

struct GmresOut {
  int iters = 0;
  bool converged = false;
};

// Flexible GMRES(m) on (L^-1 J R) y = rhs with rhs = sign * W (W = L^-1 F, sign = -1),
// right-preconditioned; the directions Z_j are unscaled state increments, so
// dX = sum_j y_j Z_j.  With c->adj the same loop solves the transposed system
// (R J^T L^-1) y = W with the transposed preconditioner (sign = +1).
GmresOut fgmres(jfnk_ctx* c, const double* X, double beta0, double sign) {
  const jfnk_opts& o = c->opts;
  hipStream_t s = c->stream;
  const size_t n = c->n;
  const int m = o.gmres_m;
  GmresOut out;
  const double target = o.gmres_eta * beta0;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  auto Hx = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
  launch_fill(n, 0.0, c->dX, s);
  bool first = true;
  while (out.iters < o.gmres_maxit) {
    double beta;
    if (first) {
      beta = beta0;
      // V_0 = sign W / beta
      launch_fill(n, 0.0, c->V, s);
      launch_axpy(n, sign / beta, c->W, c->V, s);
    } else {
      // r = sign W - A dX
      phase_begin(c);
      apply_J(c, X, c->dX, c->W2);
      phase_end(c, PH_JV);
      launch_fill(n, 0.0, c->V, s);
      launch_axpy(n, sign, c->W, c->V, s);
      launch_axpy(n, -1.0, c->W2, c->V, s);
      launch_dot<double>(n, c->V, c->V, c->scal + S_TMP, c->red, s);
      pull(c, S_TMP, 1);
      beta = std::sqrt(c->hscal[S_TMP]);
      if (!std::isfinite(beta)) throw FiniteErr("non-finite GMRES residual");
      if (beta < target) {
        out.converged = true;
        break;
      }
      launch_scale_by_inv_sqrt(n, c->V, c->scal + S_TMP, c->V, s);
    }
    first = false;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    double res = beta;
    // Arnoldi with delayed reorthogonalisation: step j orthogonalises w = A z_j once against
    // V_0..V_j and, in the same two passes, reorthogonalises V_j (orthogonalised once in
    // step j - 1) against V_0..V_{j-1}.  Column j - 1 of H is then corrected for the change of
    // V_j and its Givens rotation recomputed; the residual estimate of step j uses the
    // once-orthogonalised norm of w (the correction is of the order of rounding).
    double hprev = 0.0;                // norm of w of step j - 1 (V_j = w / hprev)
    // With the physics-based preconditioner on the forward system, V_{j+1} is left as w and read
    // as w / ||w|| by its consumers (the preconditioner's input kernels and the next step's two
    // passes, which store it normalised): one pass over the vector fewer per step, same numbers
    const bool keep_raw = !c->adj && o.precond != JFNK_PC_NONE;
    const double* vn2 = nullptr;       // slot j unnormalised: its squared norm
    std::vector<double> hcol(m + 1);   // unrotated column j - 1
    double gsave = 0.0;                // g[j - 1] before the provisional rotation j - 1
    for (int j = 0; j < m; ++j) {
      double* Vj = c->V + (size_t)j * n;
      double* Zj = c->Z + (size_t)j * n;
      double* w = c->V + (size_t)(j + 1) * n;
      phase_begin(c);
      if (c->adj) precond_T(c, X, Vj, 1, Zj);
      else precond(c, X, Vj, 1, Zj, c->opts.jv_mode == JFNK_JV_FD, vn2);
      phase_end(c, PH_PREC);
      phase_begin(c);
      apply_J(c, X, Zj, w);
      phase_end(c, PH_JV);
      const int K = j + 1;
      phase_begin(c);
      launch_dcgs2_dots(n, c->V, n, K, w, c->scal + S_H1, c->red, s, vn2);
      launch_dcgs2_update(n, c->V, n, K, c->scal + S_H1, w, w, c->scal + S_NRM3, c->red, s, vn2);
      vn2 = nullptr;
      phase_end(c, PH_ORTH);
      pull(c, S_H1, S_NRM3 + 1 - S_H1);
      const double* sums = c->hscal + S_H1;
      double hn2 = c->hscal[S_NRM3];
      if (!std::isfinite(hn2)) throw FiniteErr("non-finite Arnoldi vector");
      // the coefficients of the device's second pass
      double ss = 0.0, sb = 0.0;
      for (int i = 0; i < j; ++i) {
        ss += sums[i] * sums[i];
        sb += sums[i] * sums[K + i];
      }
      const double nu = (j == 0) ? 1.0 : std::sqrt(sums[j] - ss);
      if (!(nu > 0.0) || !std::isfinite(nu)) throw FiniteErr("loss of orthogonality in the Arnoldi basis");
      const double inv_nu = 1.0 / nu;
      if (j > 0) {
        // V_j = hprev^-1 w_prev was replaced by (V_j - sum s_i V_i) / nu: column j - 1 gains
        // hprev s_i in rows i < j and hprev nu in row j; redo its rotation
        for (int i = 0; i < j; ++i) hcol[i] += hprev * sums[i];
        hcol[j] = hprev * nu;
        for (int i = 0; i <= j; ++i) Hx(i, j - 1) = hcol[i];
        for (int i = 0; i < j - 1; ++i) {
          double t = cs[i] * Hx(i, j - 1) + sn[i] * Hx(i + 1, j - 1);
          Hx(i + 1, j - 1) = -sn[i] * Hx(i, j - 1) + cs[i] * Hx(i + 1, j - 1);
          Hx(i, j - 1) = t;
        }
        givens(Hx(j - 1, j - 1), Hx(j, j - 1), &cs[j - 1], &sn[j - 1]);
        Hx(j - 1, j - 1) = cs[j - 1] * Hx(j - 1, j - 1) + sn[j - 1] * Hx(j, j - 1);
        Hx(j, j - 1) = 0.0;
        g[j] = -sn[j - 1] * gsave;
        g[j - 1] = cs[j - 1] * gsave;
      }
      double hn = std::sqrt(hn2);
      for (int i = 0; i < j; ++i) hcol[i] = sums[K + i];
      hcol[j] = (sums[K + j] - sb) * inv_nu;
      hcol[j + 1] = hn;
      for (int i = 0; i <= j + 1; ++i) Hx(i, j) = hcol[i];
      hprev = hn;
      if (hn > 0.0) {
        if (keep_raw) {
          vn2 = c->scal + S_NRM3;
        } else {
          phase_begin(c);
          launch_scale_by_inv_sqrt(n, w, c->scal + S_NRM3, w, s);
          phase_end(c, PH_ORTH);
        }
      }
      for (int i = 0; i < j; ++i) {
        double t = cs[i] * Hx(i, j) + sn[i] * Hx(i + 1, j);
        Hx(i + 1, j) = -sn[i] * Hx(i, j) + cs[i] * Hx(i + 1, j);
        Hx(i, j) = t;
      }
      gsave = g[j];
      givens(Hx(j, j), Hx(j + 1, j), &cs[j], &sn[j]);
      Hx(j, j) = cs[j] * Hx(j, j) + sn[j] * Hx(j + 1, j);
      Hx(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      res = std::fabs(g[j + 1]);
      out.iters++;
      k = j + 1;
      if (hn == 0.0 || res < target || out.iters >= o.gmres_maxit) break;
    }
    for (int i = k - 1; i >= 0; --i) {
      double t = g[i];
      for (int l = i + 1; l < k; ++l) t -= Hx(i, l) * y[l];
      // a zero pivot follows an exact breakdown with a singular Hessenberg block
      if (Hx(i, i) == 0.0) throw FiniteErr("singular Hessenberg matrix in GMRES");
      y[i] = t / Hx(i, i);
      if (!std::isfinite(y[i])) throw FiniteErr("non-finite GMRES coefficient");
    }
    for (int i = 0; i < k; ++i) c->hscal[S_Y + i] = y[i];
    push(c, S_Y, k);
    launch_lincomb(n, c->Z, n, k, c->scal + S_Y, c->W2, s);
    launch_axpy(n, 1.0, c->W2, c->dX, s);
    check_launch();
    if (res < target) {
      out.converged = true;
      break;
    }
  }
  return out;
}

void set_state(jfnk_ctx* c, const double* Xn, double dt) {
  if (!(dt > 0.0)) throw InvErr("dt must be positive");
  c->dt = dt;
  copy_d2d(c, c->Xn, Xn, c->n * sizeof(double));
  ResidArgs a;
  a.X = c->Xn;
  a.out = c->bn;
  a.cU = 1.0 / dt;
  a.cR = 1.0 - c->prob.theta;
  launch_resid(c->G, a, 0, c->stream);
  check_launch();
  c->have_state = true;
}

int implicit_step(jfnk_ctx* c, double* X, double dt, jfnk_step_stats* st) {
  const jfnk_opts& o = c->opts;
  const Grid& G = c->G;
  hipStream_t s = c->stream;
  jfnk_step_stats S{};
  S.dt = dt;
  phase_start(c);
  set_state(c, X, dt);
  c->cg_its = 0;
  int status = JFNK_E_NEWTON_NOCONV;
  for (int k = 0; k < o.newton_max; ++k) {
    phase_begin(c);
    // W = L^-1 F(X), G0 = U/dt - theta R
    ResidArgs a;
    a.X = X;
    a.B = c->bn;
    a.out = c->W;
    a.G0 = c->G0;
    a.cU = 1.0 / dt;
    a.cR = -c->prob.theta;
    a.scaleL = 1;
    a.alpha1 = o.alpha1;
    launch_resid(G, a, 0, s);
    launch_dot<double>(c->n, c->W, c->W, c->scal + S_FN2, c->red, s);
    if (o.jv_mode == JFNK_JV_FD) launch_scaled_norm2(G, X, X, o.alpha2, c->scal + S_XN2, c->red, s);
    phase_end(c, PH_RESID);
    pull(c, S_FN2, 1);
    double fn = std::sqrt(c->hscal[S_FN2]);
    if (!std::isfinite(fn)) throw FiniteErr("non-finite residual norm");
    if (k == 0) S.f0_norm = fn;
    S.f_norm = fn;
    double dxmax = 0.0;
    if (fn > 0.0) {
      if (o.precond != JFNK_PC_NONE) {
        phase_begin(c);
        ell_setup(c, X, c->prob.theta * dt);
        phase_end(c, PH_PREC);
      }
      GmresOut go = fgmres(c, X, fn, -1.0);
      S.gmres_its += go.iters;
      launch_newton_check(G, X, c->dX, o.alpha2, 1.0, c->scal + S_DXMAX, c->red, s);
      launch_axpy(c->n, 1.0, c->dX, X, s);
      pull(c, S_DXMAX, 2);
      dxmax = c->hscal[S_DXMAX];
      if (!std::isfinite(dxmax)) throw FiniteErr("non-finite Newton correction");
      if (!(c->hscal[S_ADM] < 0.0))
        throw AdmissErr("the Newton correction gives a state with rho <= 0 or e <= 0 (no line search)");
    }
    S.newton_its = k + 1;
    S.last_dx_norm = dxmax;
    if (dxmax < o.newton_tol && k + 1 >= o.newton_min) {
      S.converged = 1;
      status = JFNK_OK;
      break;
    }
  }
  S.cg_its = c->cg_its;
  phase_finish(c, &S);
  if (st) *st = S;
  if (status != JFNK_OK) c->err = "Newton did not converge within newton_max iterations";
  return status;
}

// One step of the semi-implicit scheme used as a time stepper (Sect. 3.6):
// X^{n+1} = X^n - M^-1 F(X^n) with F(X^n) = -R(X^n), M^-1 the physics-based preconditioner
// frozen at X^n (opts.pc_schur = 1: the scheme of Sect. 3.3 with the Laplacian on p^{n+1};
// 0: the delta-form J~_V with F~_V = (dV/dU) F_U).
int si_step(jfnk_ctx* c, double* X, double dt, jfnk_step_stats* st) {
  const jfnk_opts& o = c->opts;
  const Grid& G = c->G;
  hipStream_t s = c->stream;
  if (o.precond == JFNK_PC_NONE) throw InvErr("the semi-implicit step needs a physics-based preconditioner");
  jfnk_step_stats S{};
  S.dt = dt;
  set_state(c, X, dt);
  c->cg_its = 0;
  ResidArgs a;
  a.X = X;
  a.B = c->bn;
  a.out = c->W;
  a.cU = 1.0 / dt;
  a.cR = -c->prob.theta;
  launch_resid(G, a, 0, s);
  launch_dot<double>(c->n, c->W, c->W, c->scal + S_FN2, c->red, s);
  pull(c, S_FN2, 1);
  S.f0_norm = S.f_norm = std::sqrt(c->hscal[S_FN2]);
  if (!std::isfinite(S.f0_norm)) throw FiniteErr("non-finite residual norm");
  ell_setup(c, X, si_dt(c));
  precond(c, X, c->W, 0, c->dX);
  launch_newton_check(G, X, c->dX, o.alpha2, -1.0, c->scal + S_DXMAX, c->red, s);
  launch_axpy(c->n, -1.0, c->dX, X, s);
  pull(c, S_DXMAX, 2);
  S.last_dx_norm = c->hscal[S_DXMAX];
  if (!std::isfinite(S.last_dx_norm)) throw FiniteErr("non-finite semi-implicit update");
  if (!(c->hscal[S_ADM] < 0.0))
    throw AdmissErr("the semi-implicit update gives a state with rho <= 0 or e <= 0");
  S.cg_its = c->cg_its;
  S.converged = 1;
  if (st) *st = S;
  return JFNK_OK;
}

// Adjoint of one implicit step: lam solves J^T lam = gbar at X^{n+1}; returns
// dL/dX^n = (dU/dX|_{X^n})^T lam / dt + (1 - theta) (dR/dX|_{X^n})^T lam.
struct AdjGuard {
  jfnk_ctx* c;
  explicit AdjGuard(jfnk_ctx* cc) : c(cc) { c->adj = true; }
  ~AdjGuard() { c->adj = false; }
};

int adjoint_step(jfnk_ctx* c, const double* Xn1, const double* Xn, double dt, const double* gbar,
                 double* gbar_n, jfnk_step_stats* st) {
  const jfnk_opts& o = c->opts;
  const Grid& G = c->G;
  hipStream_t s = c->stream;
  if (!(dt > 0.0)) throw InvErr("dt must be positive");
  jfnk_step_stats S{};
  S.dt = dt;
  c->dt = dt;
  c->cg_its = 0;
  phase_start(c);
  int status = JFNK_OK;
  // rhs of the scaled transposed system: R gbar (R at X^{n+1})
  launch_scale_LR(G, Xn1, o.alpha2, 1, gbar, c->W, 1, s);
  launch_dot<double>(c->n, c->W, c->W, c->scal + S_FN2, c->red, s);
  pull(c, S_FN2, 1);
  double bn = std::sqrt(c->hscal[S_FN2]);
  if (!std::isfinite(bn)) throw FiniteErr("non-finite adjoint seed");
  S.f0_norm = bn;
  if (bn == 0.0) {
    launch_fill(c->n, 0.0, c->dX, s);
    S.converged = 1;
  } else {
    AdjGuard guard(c);
    if (o.precond != JFNK_PC_NONE) ell_setup(c, Xn1, c->prob.theta * dt);
    GmresOut go = fgmres(c, Xn1, bn, 1.0);
    S.gmres_its = go.iters;
    S.converged = go.converged ? 1 : 0;
    if (!go.converged) {
      status = JFNK_E_GMRES_NOCONV;
      c->err = "adjoint GMRES did not reach gmres_eta within gmres_maxit iterations";
    }
  }
  // dL/dX^n from lam (in dX)
  launch_vjp(G, Xn, c->dX, 1.0 / dt, 1.0 - c->prob.theta, c->vjps, 0, o.alpha2, gbar_n, s);
  check_launch();
  S.newton_its = 0;
  S.cg_its = c->cg_its;
  phase_finish(c, &S);
  if (st) *st = S;
  return status;
}

void destroy_bufs(jfnk_ctx* c) {
  for (auto& e : c->pev)
    if (e) (void)hipEventDestroy(e);
  for (void* p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
  if (c->hscal) (void)hipHostFree(c->hscal);
  c->hscal = nullptr;
  if (c->hctl) (void)hipHostFree(c->hctl);
  c->hctl = nullptr;
}

void create(jfnk_ctx* c) {
  const Grid& G = c->G;
  c->nvar = 2 + G.nd;
  c->n = (size_t)c->nvar * G.N;
  c->m_alloc = c->opts.gmres_m;
  size_t n = c->n;
  c->bn = dalloc<double>(c, n);
  c->Xn = dalloc<double>(c, n);
  c->G0 = dalloc<double>(c, n);
  c->W = dalloc<double>(c, n);
  c->W2 = dalloc<double>(c, n);
  c->dX = dalloc<double>(c, n);
  c->Xk = dalloc<double>(c, n);
  c->V = dalloc<double>(c, n * (c->m_alloc + 1));
  c->Z = dalloc<double>(c, n * c->m_alloc);
  c->scal = dalloc<double>(c, S_COUNT);
  HIPX(hipHostMalloc((void**)&c->hscal, S_COUNT * sizeof(double), hipHostMallocDefault));
  std::memset(c->hscal, 0, S_COUNT * sizeof(double));
  c->red.part = dalloc<double>(c, (size_t)kRedBlocks * 2 * kMaxK);
  c->red.count = dalloc<unsigned int>(c, 1);
  HIPX(hipMemsetAsync(c->red.count, 0, sizeof(unsigned int), c->stream));
  HIPX(hipMemsetAsync(c->scal, 0, S_COUNT * sizeof(double), c->stream));
  size_t N = (size_t)G.N;
  c->rhs_p = dalloc<double>(c, N);
  c->dp = dalloc<double>(c, N);
  c->rhs_T = dalloc<double>(c, N);
  c->dT = dalloc<double>(c, N);
  for (int i = 0; i < 7; ++i) c->cg64[i] = dalloc<double>(c, N);
  bool want32 = true;  // precision may be switched by jfnk_set_opts
  for (int i = 0; i < 9; ++i) c->cg32[i] = dalloc<float>(c, N);
  c->ctl = dalloc<CGCtl>(c, 1);
  HIPX(hipMemsetAsync(c->ctl, 0, sizeof(CGCtl), c->stream));
  c->cgpart = dalloc<double>(c, (size_t)kPartCount * kRedBlocks);
  HIPX(hipHostMalloc((void**)&c->hctl, sizeof(CGCtl), hipHostMallocDefault));
  std::memset(c->hctl, 0, sizeof(CGCtl));
  c->zero64 = dalloc<double>(c, 1);
  c->zero32 = dalloc<float>(c, 1);
  HIPX(hipMemsetAsync(c->zero64, 0, sizeof(double), c->stream));
  HIPX(hipMemsetAsync(c->zero32, 0, sizeof(float), c->stream));
  build_hierarchy(c, c->ops[0], want32);
  build_hierarchy(c, c->ops[1], want32);
  c->vjps = dalloc<double>(c, vjp_scratch_doubles(G));
  sync(c);
}

}  // namespace

// ======================================================================================
// C ABI
// ======================================================================================
#define ABI_BEGIN try {
#define ABI_END(ctx)                                                             \
  }                                                                              \
  catch (const InvErr& e) {                                                      \
    (ctx)->err = e.msg;                                                          \
    return JFNK_E_INVALID;                                                       \
  }                                                                              \
  catch (const DevErr& e) {                                                      \
    (ctx)->err = e.msg;                                                          \
    return JFNK_E_DEVICE;                                                        \
  }                                                                              \
  catch (const FiniteErr& e) {                                                   \
    (ctx)->err = e.msg;                                                          \
    return JFNK_E_NONFINITE;                                                     \
  }                                                                              \
  catch (const AdmissErr& e) {                                                   \
    (ctx)->err = e.msg;                                                          \
    return JFNK_E_INADMISSIBLE;                                                  \
  }                                                                              \
  catch (...) {                                                                  \
    (ctx)->err = "unexpected host exception";                                    \
    return JFNK_E_DEVICE;                                                        \
  }

extern "C" {

void jfnk_default_opts(jfnk_opts* o) {
  if (!o) return;
  o->newton_tol = 1e-8;
  o->newton_max = 20;
  o->newton_min = 2;
  o->gmres_m = 30;
  o->gmres_maxit = 300;
  o->gmres_eta = 1e-4;
  o->jv_mode = JFNK_JV_FD;
  o->fd_lambda = 1e-7;
  o->alpha1 = 1e-5;
  o->alpha2 = 1.0;
  o->precond = JFNK_PC_SOUND;
  o->ell_precision = JFNK_FP64;
  o->cg_eta = 1e-4;
  o->cg_maxit = 50;
  o->pc_schur = 0;
  o->phase_timing = 0;
  o->mg_levels = 0;
  o->mg_smooth = 2;
}

int jfnk_create(const jfnk_problem* prob, const jfnk_opts* opts, void* hip_stream, jfnk_ctx** out) {
  if (!out) return JFNK_E_INVALID;
  *out = nullptr;
  jfnk_ctx* c = new (std::nothrow) jfnk_ctx();
  if (!c) return JFNK_E_DEVICE;
  try {
    validate(prob, opts);
    c->prob = *prob;
    c->opts = *opts;
    c->G = make_grid(*prob);
    c->stream = (hipStream_t)hip_stream;
    create(c);
  } catch (const InvErr& e) {
    g_create_err = e.msg;
    destroy_bufs(c);
    delete c;
    return JFNK_E_INVALID;
  } catch (const DevErr& e) {
    g_create_err = e.msg;
    destroy_bufs(c);
    delete c;
    return JFNK_E_DEVICE;
  } catch (...) {
    g_create_err = "unexpected host exception";
    destroy_bufs(c);
    delete c;
    return JFNK_E_DEVICE;
  }
  *out = c;
  return JFNK_OK;
}

int jfnk_destroy(jfnk_ctx* c) {
  if (!c) return JFNK_E_INVALID;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  destroy_bufs(c);
  delete c;
  return JFNK_OK;
}

int jfnk_set_opts(jfnk_ctx* c, const jfnk_opts* o) {
  if (!c) return JFNK_E_INVALID;
  ABI_BEGIN
  validate(&c->prob, o);
  if (o->gmres_m > c->m_alloc) throw InvErr("gmres_m exceeds the restart length the context was created with");
  if (o->mg_levels != c->opts.mg_levels) throw InvErr("mg_levels is fixed when the context is created");
  c->opts = *o;
  return JFNK_OK;
  ABI_END(c)
}

size_t jfnk_workspace_bytes(const jfnk_ctx* c) { return c ? c->bytes : 0; }

const char* jfnk_last_error(const jfnk_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

int jfnk_set_state_n(jfnk_ctx* c, const double* Xn, double dt) {
  if (!c) return JFNK_E_INVALID;
  ABI_BEGIN
  if (!Xn) throw InvErr("null X^n");
  set_state(c, Xn, dt);
  return JFNK_OK;
  ABI_END(c)
}

int jfnk_residual(jfnk_ctx* c, const double* X, double* F) {
  if (!c) return JFNK_E_INVALID;
  ABI_BEGIN
  if (!X || !F) throw InvErr("null array");
  if (!c->have_state) throw InvErr("jfnk_set_state_n must be called first");
  ResidArgs a;
  a.X = X;
  a.B = c->bn;
  a.out = F;
  a.cU = 1.0 / c->dt;
  a.cR = -c->prob.theta;
  launch_resid(c->G, a, 0, c->stream);
  check_launch();
  return JFNK_OK;
  ABI_END(c)
}

int jfnk_jvp(jfnk_ctx* c, const double* X, const double* v, double* Jv, int32_t mode) {
  if (!c) return JFNK_E_INVALID;
  ABI_BEGIN
  if (!X || !v || !Jv) throw InvErr("null array");
  if (!c->have_state) throw InvErr("jfnk_set_state_n must be called first");
  ResidArgs a;
  a.X = X;
  a.V = v;
  a.out = Jv;
  a.cU = 1.0 / c->dt;
  a.cR = -c->prob.theta;
  if (mode == JFNK_JV_EXACT) {
    launch_resid(c->G, a, 1, c->stream);
  } else if (mode == JFNK_JV_FD) {
    ResidArgs g;
    g.X = X;
    g.out = c->G0;
    g.cU = a.cU;
    g.cR = a.cR;
    launch_resid(c->G, g, 0, c->stream);  // G0 = U/dt - theta R at X
    launch_scaled_norm2(c->G, X, X, c->opts.alpha2, c->scal + S_XN2, c->red, c->stream);
    launch_scaled_norm2(c->G, X, v, c->opts.alpha2, c->scal + S_ZN2, c->red, c->stream);
    a.B = c->G0;
    a.fd_norms = c->scal + S_XN2;
    a.fd_lambda = c->opts.fd_lambda;
    a.shift = c->Xk;
    launch_resid(c->G, a, 2, c->stream);
  } else {
    throw InvErr("bad mode");
  }
  check_launch();
  return JFNK_OK;
  ABI_END(c)
}

int jfnk_precond_apply(jfnk_ctx* c, const double* X, const double* r, double* z) {
  if (!c) return JFNK_E_INVALID;
  ABI_BEGIN
  if (!X || !r || !z) throw InvErr("null array");
  if (!c->have_state) throw InvErr("jfnk_set_state_n must be called first");
  c->cg_its = 0;
  if (c->opts.precond != JFNK_PC_NONE) ell_setup(c, X, si_dt(c));
  precond(c, X, r, 0, z);
  sync(c);
  return JFNK_OK;
  ABI_END(c)
}

int jfnk_precond_apply_transpose(jfnk_ctx* c, const double* X, const double* w, double* z) {
  if (!c) return JFNK_E_INVALID;
  ABI_BEGIN
  if (!X || !w || !z) throw InvErr("null array");
  if (!c->have_state) throw InvErr("jfnk_set_state_n must be called first");
  c->cg_its = 0;
  if (c->opts.precond != JFNK_PC_NONE) ell_setup(c, X, si_dt(c));
  precond_T(c, X, w, 0, z);
  sync(c);
  return JFNK_OK;
  ABI_END(c)
}

int jfnk_si_step(jfnk_ctx* c, double* X, double dt, jfnk_step_stats* st) {
  if (!c) return JFNK_E_INVALID;
  ABI_BEGIN
  if (!X) throw InvErr("null X");
  int r = si_step(c, X, dt, st);
  sync(c);
  return r;
  ABI_END(c)
}

int jfnk_implicit_step(jfnk_ctx* c, double* X, double dt, jfnk_step_stats* st) {
  if (!c) return JFNK_E_INVALID;
  ABI_BEGIN
  if (!X) throw InvErr("null X");
  int r = implicit_step(c, X, dt, st);
  sync(c);
  return r;
  ABI_END(c)
}

double jfnk_cfl_dt(jfnk_ctx* c, const double* X, double cfl) {
  if (!c || !X || !(cfl > 0.0)) return -1.0;
  try {
    launch_cfl_speed(c->G, X, c->scal + S_TMP, c->red, c->stream);
    pull(c, S_TMP, 1);
    double hmin = c->G.dx[0];
    for (int d = 1; d < c->G.nd; ++d) hmin = std::min(hmin, c->G.dx[d]);
    return cfl * hmin / c->hscal[S_TMP];
  } catch (const DevErr& e) {
    c->err = e.msg;
    return -1.0;
  }
}

int jfnk_vjp(jfnk_ctx* c, const double* X, const double* w, double* JTw) {
  if (!c) return JFNK_E_INVALID;
  ABI_BEGIN
  if (!X || !w || !JTw) throw InvErr("null array");
  if (!c->have_state) throw InvErr("jfnk_set_state_n must be called first");
  launch_vjp(c->G, X, w, 1.0 / c->dt, -c->prob.theta, c->vjps, 0, c->opts.alpha2, JTw, c->stream);
  check_launch();
  return JFNK_OK;
  ABI_END(c)
}

int jfnk_vjp_prev(jfnk_ctx* c, const double* Xn, const double* lam, double* out) {
  if (!c) return JFNK_E_INVALID;
  ABI_BEGIN
  if (!Xn || !lam || !out) throw InvErr("null array");
  if (!c->have_state) throw InvErr("jfnk_set_state_n must be called first");
  launch_vjp(c->G, Xn, lam, -1.0 / c->dt, -(1.0 - c->prob.theta), c->vjps, 0, c->opts.alpha2, out,
             c->stream);
  check_launch();
  return JFNK_OK;
  ABI_END(c)
}

int jfnk_probe_enable(int32_t on) {
  probe_enable(on != 0);
  return JFNK_OK;
}

int jfnk_probe_count(void) { return KF_COUNT; }

const char* jfnk_probe_name(int32_t k) { return (k >= 0 && k < KF_COUNT) ? kFamNames[k] : ""; }

int jfnk_probe_read(int32_t k, double* ms, int64_t* launches, double* bytes) {
  if (!ms || !launches || !bytes) return JFNK_E_INVALID;
  long long n = 0;
  if (!probe_read(k, ms, &n, bytes)) return JFNK_E_INVALID;
  *launches = n;
  return JFNK_OK;
}

int jfnk_adjoint_step(jfnk_ctx* c, const double* Xn1, const double* Xn, double dt,
                      const double* gbar_n1, double* gbar_n, jfnk_step_stats* st) {
  if (!c) return JFNK_E_INVALID;
  ABI_BEGIN
  if (!Xn1 || !Xn || !gbar_n1 || !gbar_n) throw InvErr("null array");
  int r = adjoint_step(c, Xn1, Xn, dt, gbar_n1, gbar_n, st);
  sync(c);
  return r;
  ABI_END(c)
}

}  // extern "C"

