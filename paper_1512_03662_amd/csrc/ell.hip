// Physics-based preconditioner kernels (Sect. 4.3 with the semi-implicit schemes of
// Sects. 3.3-3.4) and the multigrid-preconditioned CG used for its parabolic systems
// (Sect. 3.5 solves them with a preconditioned Krylov method to eta').
//
// Elliptic operators (cell-centred, 5/7-point, symmetric positive definite):
//   pressure  A_p = diag(1/(Gamma1 p dt)) - dt div_h(rho_f^-1 grad_h)  (row-scaled by
//             1/(Gamma1 p) so that it is symmetric),
//   thermal   A_T = diag(rho c_v/dt) - div_h(chi_f grad_h)   (dT = de/c_v, Sect. 3.4),
// stored as a diagonal and one weight per low face; wall faces carry weight 0.
// Multigrid: coarsening by 2 per axis; coarse diagonal = mean of the children, coarse face
// weight = mean of the covered fine weights / 4; restriction = mean, prolongation =
// injection; Chebyshev-Jacobi smoothing of degree 2 on [0.5, 2] (2 bounds lambda_max(D^-1 A)
// by Gershgorin); dense inverse at the coarsest level.
#include "common.hpp"
#include "kernels.hpp"
#include "probe.hpp"

namespace jfnk {

// Chebyshev(2) coefficients on [lmin, lmax] = [0.5, 2]
constexpr double kChebTheta = 1.25;
constexpr double kChebC1 = 0.6 / (2.0 * (1.25 / 0.75) - 0.6);          // rho1 rho0
constexpr double kChebC2 = 2.0 / (2.0 * (1.25 / 0.75) - 0.6) / 0.75;   // 2 rho1 / delta

template <class T>
struct LV {
  int n[3];
  int stride[3];
  int N;
  int bc[3];
  const T* diag;
  const T* w[3];
  const T* dinv;
};

template <class T>
static LV<T> view(const Grid& G, const Level& L) {
  LV<T> v;
  for (int d = 0; d < 3; ++d) {
    v.n[d] = L.n[d];
    v.stride[d] = L.stride[d];
    v.bc[d] = G.bc[d];
    v.w[d] = (const T*)L.w[d];
  }
  v.N = L.N;
  v.diag = (const T*)L.diag;
  v.dinv = (const T*)L.dinv;
  return v;
}

template <int ND>
__device__ __forceinline__ void coords(const int* n, int lin, int* c) {
  c[0] = lin % n[0];
  int r = lin / n[0];
  c[1] = r % n[1];
  c[2] = r / n[1];
}

// (A phi)[c]; nb(d, s, k) is phi at the neighbour k (linear index, wrapped) on side s = -1/+1
// of axis d, phic = phi at c.  Neighbours across a wall are wrapped too: their face weight
// is 0.
template <class T, int ND, class F>
__device__ __forceinline__ T apply_nb(const LV<T>& L, const int* c, int lin, const F& nb, T phic) {
  T out = L.diag[lin] * phic;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const int n = L.n[d], st = L.stride[d];
    const int cm = (c[d] == 0) ? lin + (n - 1) * st : lin - st;
    const int cp = (c[d] == n - 1) ? lin - (n - 1) * st : lin + st;
    const T wl = L.w[d][lin];
    const T wu = (L.bc[d] == 1 && c[d] == n - 1) ? T(0) : L.w[d][cp];
    out -= wu * (nb(d, 1, cp) - phic) - wl * (phic - nb(d, -1, cm));
  }
  return out;
}

// (A phi)[c] with phi given by a functor of the linear index; phic = phi(lin)
template <class T, int ND, class F>
__device__ __forceinline__ T apply_at(const LV<T>& L, const int* c, int lin, const F& phi, T phic) {
  return apply_nb<T, ND>(L, c, lin, [&](int, int, int k) { return phi(k); }, phic);
}

// A's row at one cell (diagonal, face weights, neighbour indices), loaded ahead of a kernel's
// LDS phase so that its memory latency overlaps that phase; apply_row then evaluates the row
// exactly as apply_nb does
template <class T, int ND>
struct RowCoef {
  T diag, wl[3], wu[3];
  int cm[3], cp[3];
};
template <class T, int ND>
__device__ __forceinline__ RowCoef<T, ND> row_coef(const LV<T>& L, const int* c, int lin) {
  RowCoef<T, ND> r;
  r.diag = L.diag[lin];
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const int n = L.n[d], st = L.stride[d];
    r.cm[d] = (c[d] == 0) ? lin + (n - 1) * st : lin - st;
    r.cp[d] = (c[d] == n - 1) ? lin - (n - 1) * st : lin + st;
    r.wl[d] = L.w[d][lin];
    r.wu[d] = (L.bc[d] == 1 && c[d] == n - 1) ? T(0) : L.w[d][r.cp[d]];
  }
  return r;
}
template <class T, int ND, class F>
__device__ __forceinline__ T apply_row(const RowCoef<T, ND>& r, const F& nb, T phic) {
  T out = r.diag * phic;
#pragma unroll
  for (int d = 0; d < ND; ++d) out -= r.wu[d] * (nb(d, 1, r.cp[d]) - phic) - r.wl[d] * (phic - nb(d, -1, r.cm[d]));
  return out;
}

// restricted residual (mean over the 2^ND children of b - A x) of coarse cell cc; UNR
// children are unrolled at a time (the sum's order is the same)
template <class T, int ND, int UNR = (1 << ND)>
__device__ __forceinline__ T restrict_at(const LV<T>& F, const T* b, const T* x, const int* cc) {
  auto xf = [&](int i) { return x[i]; };
  T sum = T(0);
#pragma unroll UNR
  for (int ch = 0; ch < (1 << ND); ++ch) {
    int c[3] = {0, 0, 0};
    int fl = 0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      c[d] = 2 * cc[d] + ((ch >> d) & 1);
      fl += c[d] * F.stride[d];
    }
    sum += b[fl] - apply_at<T, ND>(F, c, fl, xf, x[fl]);
  }
  return sum * T(1.0 / (1 << ND));
}

// ---- coefficients ------------------------------------------------------------------------
template <int ND>
__global__ void __launch_bounds__(kBlock) k_ell_coef(Grid G, const double* X, double dt, int op, double* diag,
                                                     double* w0, double* w1, double* w2) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (lin >= G.N) return;
  Pos P = make_pos<ND>(G, lin);
  const double gm1 = G.gamma - 1.0;
  const bool rad = G.a_rad != 0.0;
  const double rho = X[lin], e = X[G.N + lin];
  double* w[3] = {w0, w1, w2};
  Thermo th{};
  if (rad) th = thermo<true>(G, rho, e);
  // pressure: 1/(Gamma1 p dt); thermal: rho c_v/dt with c_v = de/dT|_rho
  if (op == 0) {
    diag[lin] = rad ? 1.0 / (th.G1 * th.p * dt) : 1.0 / (G.gamma * gm1 * rho * e * dt);
  } else {
    diag[lin] = rad ? rho * th.cv / dt : rho / (gm1 * dt);
  }
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    double s;
    int im = gidx<ND>(G, P, 0, shift(off0(), d, -1), &s);
    double wf;
    if (G.bc[d] == 1 && P.c[d] == 0) {
      wf = 0.0;
    } else if (op == 0) {
      double rf = 0.5 * (X[im] + rho);
      wf = dt / (rf * G.dx[d] * G.dx[d]);
    } else {
      double Tm = rad ? rad_temperature(G, X[im], X[G.N + im]) : gm1 * X[G.N + im];
      double T0 = rad ? th.T : gm1 * e;
      double cm, c0;
      if (G.chi_model == 1) {
        cm = G.chi0;
        c0 = G.chi0;
      } else if (G.chi_model == 2) {
        cm = G.chi0 * powr(Tm * G.chi_tref_inv, G.chi_exp);
        c0 = G.chi0 * powr(T0 * G.chi_tref_inv, G.chi_exp);
      } else {
        cm = 0.0;
        c0 = 0.0;
      }
      wf = 0.5 * (cm + c0) / (G.dx[d] * G.dx[d]);
    }
    w[d][lin] = wf;
  }
}

void launch_ell_coef(const Grid& G, const double* X, double dt, int op, double* diag,
                     double* const* w, hipStream_t s) {
  dim3 gr((G.N + kBlock - 1) / kBlock);
  if (G.nd == 2) k_ell_coef<2><<<gr, kBlock, 0, s>>>(G, X, dt, op, diag, w[0], w[1], nullptr);
  else k_ell_coef<3><<<gr, kBlock, 0, s>>>(G, X, dt, op, diag, w[0], w[1], w[2]);
}

template <class T, int ND>
__global__ void __launch_bounds__(kBlock) k_ell_coarsen(Level f, Level c) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (lin >= c.N) return;
  int cc[3];
  coords<ND>(c.n, lin, cc);
  const T* fd = (const T*)f.diag;
  int base = 0;
#pragma unroll
  for (int d = 0; d < ND; ++d) base += 2 * cc[d] * f.stride[d];
  // diagonal: mean of the 2^ND children
  double sdiag = 0.0;
#pragma unroll
  for (int ch = 0; ch < (1 << ND); ++ch) {
    int off = 0;
#pragma unroll
    for (int d = 0; d < ND; ++d) off += ((ch >> d) & 1) * f.stride[d];
    sdiag += (double)fd[base + off];
  }
  ((T*)c.diag)[lin] = (T)(sdiag / (1 << ND));
  // face weights: mean of the 2^(ND-1) covered fine faces, / 4
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const T* fw = (const T*)f.w[d];
    double sw = 0.0;
#pragma unroll
    for (int ch = 0; ch < (1 << ND); ++ch) {
      if ((ch >> d) & 1) continue;  // only children on the low-d side
      int off = 0;
#pragma unroll
      for (int e = 0; e < ND; ++e) off += ((ch >> e) & 1) * f.stride[e];
      sw += (double)fw[base + off];
    }
    ((T*)c.w[d])[lin] = (T)(sw / (1 << (ND - 1)) / 4.0);
  }
}

template <class T>
void launch_ell_coarsen(const Grid& G, const Level& f, const Level& c, hipStream_t s) {
  dim3 gr((c.N + kBlock - 1) / kBlock);
  if (G.nd == 2) k_ell_coarsen<T, 2><<<gr, kBlock, 0, s>>>(f, c);
  else k_ell_coarsen<T, 3><<<gr, kBlock, 0, s>>>(f, c);
}

template <class T, int ND>
__global__ void __launch_bounds__(kBlock) k_ell_dinv(LV<T> L, T* dinv) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (lin >= L.N) return;
  int c[3];
  coords<ND>(L.n, lin, c);
  double D = (double)L.diag[lin];
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const int n = L.n[d], st = L.stride[d];
    const int cp = (c[d] == n - 1) ? lin - (n - 1) * st : lin + st;
    double wu = (L.bc[d] == 1 && c[d] == n - 1) ? 0.0 : (double)L.w[d][cp];
    D += (double)L.w[d][lin] + wu;
  }
  dinv[lin] = (T)(1.0 / D);
}

template <class T>
void launch_ell_dinv(const Grid& G, const Level& L, hipStream_t s) {
  dim3 gr((L.N + kBlock - 1) / kBlock);
  LV<T> v = view<T>(G, L);
  if (G.nd == 2) k_ell_dinv<T, 2><<<gr, kBlock, 0, s>>>(v, (T*)L.dinv);
  else k_ell_dinv<T, 3><<<gr, kBlock, 0, s>>>(v, (T*)L.dinv);
}

__global__ void k_to_f32(int n, const double* a, float* b) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}
void launch_level_to_f32(const Level& src, const Level& dst, int nd, hipStream_t s) {
  dim3 gr((src.N + kBlock - 1) / kBlock);
  k_to_f32<<<gr, kBlock, 0, s>>>(src.N, (const double*)src.diag, (float*)dst.diag);
  k_to_f32<<<gr, kBlock, 0, s>>>(src.N, (const double*)src.dinv, (float*)dst.dinv);
  for (int d = 0; d < nd; ++d)
    k_to_f32<<<gr, kBlock, 0, s>>>(src.N, (const double*)src.w[d], (float*)dst.w[d]);
}

// ---- CG control and partial sums --------------------------------------------------------
// A CG solve is driven from the device: every kernel of an iteration returns at once when
// the control block's flag is set, so the host enqueues iterations ahead of the test.
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of n partials in a fixed order; every block of a launch obtains the same value.
__device__ double block_sum_parts(const double* P, int n) {
  __shared__ double sm[kCoarseThreads / 64];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v += P[i];
  v = wave_sum_d(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) sm[wid] = v;
  __syncthreads();
  double a = sm[0];
  for (int w = 1; w < nw; ++w) a += sm[w];
  __syncthreads();
  return a;
}

// P[blockIdx.x] = sum of v over the block
__device__ void block_partial(double v, double* P) {
  __shared__ double sm[kCoarseThreads / 64];
  v = wave_sum_d(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) sm[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = sm[0];
    for (int w = 1; w < nw; ++w) a += sm[w];
    P[blockIdx.x] = a;
  }
}

// convergence test of iteration it: ||r|| < eta ||b||, or the iteration limit
__device__ void cg_decide(const CGArgs& g, double rr, int it) {
  CGCtl* S = g.ctl;
  S->rr = rr;
  const double rn = sqrt(rr), bn = sqrt(S->bb);
  if (!isfinite(rn)) {
    S->its = it;
    S->flag = -1;
  } else if (rn < g.eta * bn || it >= g.maxit) {
    S->its = it;
    S->flag = 1;
  }
}

static inline int red_grid(size_t n) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > (size_t)kRedBlocks) b = kRedBlocks;
  return (int)(b < 1 ? 1 : b);
}

int cg_partials(size_t n) { return red_grid(n); }

// cells of a launch: one per thread when the grid covers N, grid-stride otherwise
#define FOR_CELLS(lin, N) \
  for (int lin = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; lin < (N); lin += gridDim.x * kBlock)

// ---- V-cycle pieces ------------------------------------------------------------------------
// INIT: first smoothing of a solve; also resets the control block and writes the (b, b)
// partials
template <class T, int ND, bool INIT>
__global__ void __launch_bounds__(kBlock) k_mg_presmooth(LV<T> L, const T* b, T* x, CGArgs g) {
  if (INIT) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      g.ctl->flag = 0;
      g.ctl->its = 0;
    }
  } else if (g.ctl->flag) {
    return;
  }
  const T th = T(1.0 / kChebTheta);
  T acc = T(0);
  FOR_CELLS(lin, L.N) {
    int c[3];
    coords<ND>(L.n, lin, c);
    auto x1 = [&](int i) { return L.dinv[i] * b[i] * th; };
    T x1c = x1(lin);
    T Ax = apply_at<T, ND>(L, c, lin, x1, x1c);
    x[lin] = (T(1.0) + T(kChebC1)) * x1c + T(kChebC2) * L.dinv[lin] * (b[lin] - Ax);
    if (INIT) acc += b[lin] * b[lin];
  }
  if (INIT) block_partial((double)acc, g.part + kPartBB * kRedBlocks);
}

// CONV: block 0 also takes the convergence decision of iteration it from the (r, r) partials
// (the other blocks of this launch may or may not see it; their output is then unused)
template <class T, int ND, bool CONV>
__global__ void __launch_bounds__(kBlock) k_mg_restrict_resid(LV<T> L, const T* b, const T* x, T* bc,
                                                              int Nc, int nc0, int nc1, CGArgs g, int it) {
  if (g.ctl->flag) return;
  if (CONV && blockIdx.x == 0) {
    const double rr = block_sum_parts(g.part + kPartRR * kRedBlocks, g.np);
    if (threadIdx.x == 0) cg_decide(g, rr, it);
  }
  auto xf = [&](int i) { return x[i]; };
  FOR_CELLS(lin, Nc) {
    int cc[3];
    cc[0] = lin % nc0;
    int r = lin / nc0;
    cc[1] = r % nc1;
    cc[2] = r / nc1;
    T sum = T(0);
#pragma unroll
    for (int ch = 0; ch < (1 << ND); ++ch) {
      int c[3] = {0, 0, 0};
      int fl = 0;
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        c[d] = 2 * cc[d] + ((ch >> d) & 1);
        fl += c[d] * L.stride[d];
      }
      sum += b[fl] - apply_at<T, ND>(L, c, fl, xf, x[fl]);
    }
    bc[lin] = sum * T(1.0 / (1 << ND));
  }
}

template <class T, int ND>
__device__ __forceinline__ int parent_of(const LV<T>& L, int lin, const int* cstride) {
  int c[3];
  coords<ND>(L.n, lin, c);
  int p = 0;
#pragma unroll
  for (int d = 0; d < ND; ++d) p += (c[d] >> 1) * cstride[d];
  return p;
}

template <class T, int ND>
__global__ void __launch_bounds__(kBlock) k_mg_prolong_smooth1(LV<T> L, const T* b, const T* x2, const T* xc,
                                                               int cs0, int cs1, int cs2, T* x1, T* d0,
                                                               CGArgs g) {
  if (g.ctl->flag) return;
  const int cst[3] = {cs0, cs1, cs2};
  auto xp = [&](int i) { return x2[i] + xc[parent_of<T, ND>(L, i, cst)]; };
  FOR_CELLS(lin, L.N) {
    int c[3];
    coords<ND>(L.n, lin, c);
    T xpc = xp(lin);
    T r0 = b[lin] - apply_at<T, ND>(L, c, lin, xp, xpc);
    T dd = L.dinv[lin] * r0 * T(1.0 / kChebTheta);
    x1[lin] = xpc + dd;
    d0[lin] = dd;
  }
}

// RZ: also the (b, x) partials (b the level's right-hand side, x the result)
template <class T, int ND, bool RZ>
__global__ void __launch_bounds__(kBlock) k_mg_smooth2(LV<T> L, const T* b, const T* x1, const T* d0, T* x,
                                                       CGArgs g) {
  if (g.ctl->flag) return;
  auto xf = [&](int i) { return x1[i]; };
  T acc = T(0);
  FOR_CELLS(lin, L.N) {
    int c[3];
    coords<ND>(L.n, lin, c);
    T x1c = x1[lin];
    T r1 = b[lin] - apply_at<T, ND>(L, c, lin, xf, x1c);
    T xn = x1c + T(kChebC1) * d0[lin] + T(kChebC2) * L.dinv[lin] * r1;
    x[lin] = xn;
    if (RZ) acc += b[lin] * xn;
  }
  if (RZ) block_partial((double)acc, g.part + kPartRZ * kRedBlocks);
}

// ---- z-marching forms of the single-level kernels on 3D grids ---------------------------
// A block owns kZX x kZY columns of cells (x contiguous) and walks them along z through a
// chunk of planes.  Fields that a kernel reads or writes once per cell (right-hand sides,
// diagonals, smoother corrections, CG updates) go through non-temporal loads and stores, so
// that they do not displace the stencil operand's neighbouring rows from the caches.  The state a cell's stencil needs from its z neighbours is carried in
// registers from one plane to the next, so no plane is fetched a second time for the z+1 or
// z-1 neighbour of another cell (the grid-stride forms read those planes again, from another
// XCD's L2 or from memory).  Except for the restriction, which has a grid of its own, a
// launch has exactly cg_partials(N) blocks (one partial each where the kernel writes
// partials); blocks past the last chunk have no cells.
constexpr int kZX = 64, kZY = 4;
static_assert(kZX * kZY == kBlock, "one cell column per thread");

struct ZChunk {
  int cx, cy, z0, z1;  // the thread's column and its planes [z0, z1); z0 >= z1: no cells
};
__device__ __forceinline__ ZChunk zchunk(const int* n, int zc) {
  const int nbx = (n[0] + kZX - 1) / kZX, nby = (n[1] + kZY - 1) / kZY;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int tile = b % (nbx * nby), chunk = b / (nbx * nby);
  ZChunk z;
  z.cx = (tile % nbx) * kZX + (int)threadIdx.x % kZX;
  z.cy = (tile / nbx) * kZY + (int)threadIdx.x / kZX;
  z.z0 = chunk * zc;
  z.z1 = min(z.z0 + zc, n[2]);
  if (z.cx >= n[0] || z.cy >= n[1]) z.z1 = z.z0;
  return z;
}

// Walks the thread's column: st(i, x, y, z) is the per-cell state at cell i (coordinates
// x, y, z), val(state) the value the stencil applies A to; emit(lin, z, state, A val) is
// called for every cell of the chunk in increasing z.  The row is evaluated in apply_nb's
// order, with the z neighbours' values and the upper z face weight taken from the carried
// planes.
template <class T, class St, class Val, class Emit>
__device__ __forceinline__ void zmarch(const LV<T>& L, const ZChunk& zc, const St& st, const Val& val,
                                       const Emit& emit) {
  if (zc.z0 >= zc.z1) return;
  const int nz = L.n[2], sz = L.stride[2];
  const int col = zc.cx + zc.cy * L.stride[1];
  const int c[2] = {zc.cx, zc.cy};
  int lin = col + zc.z0 * sz;
  const int zm0 = (zc.z0 == 0) ? nz - 1 : zc.z0 - 1;
  auto vm = val(st(col + zm0 * sz, zc.cx, zc.cy, zm0));
  auto sc = st(lin, zc.cx, zc.cy, zc.z0);
  T w2c = L.w[2][lin];
  for (int z = zc.z0; z < zc.z1; ++z, lin += sz) {
    const int zn = (z == nz - 1) ? 0 : z + 1;
    const int ln = col + zn * sz;
    const auto sn = st(ln, zc.cx, zc.cy, zn);
    const T w2n = L.w[2][ln];
    const T pc = val(sc);
    T out = __builtin_nontemporal_load(&L.diag[lin]) * pc;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int n = L.n[d], s = L.stride[d];
      const int cm = (c[d] == 0) ? lin + (n - 1) * s : lin - s;
      const int cp = (c[d] == n - 1) ? lin - (n - 1) * s : lin + s;
      int qm[2] = {c[0], c[1]}, qp[2] = {c[0], c[1]};
      qm[d] = (c[d] == 0) ? n - 1 : c[d] - 1;
      qp[d] = (c[d] == n - 1) ? 0 : c[d] + 1;
      const T wl = L.w[d][lin];
      const T wu = (L.bc[d] == 1 && c[d] == n - 1) ? T(0) : L.w[d][cp];
      out -= wu * (val(st(cp, qp[0], qp[1], z)) - pc) - wl * (pc - val(st(cm, qm[0], qm[1], z)));
    }
    {
      const T wu = (L.bc[2] == 1 && z == nz - 1) ? T(0) : w2n;
      out -= wu * (val(sn) - pc) - w2c * (pc - vm);
    }
    emit(lin, z, sc, out);
    vm = pc;
    sc = sn;
    w2c = w2n;
  }
}

template <class T>
struct UpdSt {
  T r, dv, x1;  // new residual, inverse diagonal, first smoothing iterate
};

// k_cg_update<T, 3, true> in z-marching form
template <class T>
__global__ void __launch_bounds__(kBlock) k_cg_update_zm(LV<T> L, const T* rold, const T* q, const T* p, T* x,
                                                         T* rnew, T* xm, CGArgs g, int it, int zc) {
  CGCtl* S = g.ctl;
  if (S->flag) return;
  if (it == 1 && S->bb == 0.0) {  // b = 0: x = 0 was written by the apply kernel
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      S->its = 0;
      S->flag = 1;
    }
    return;
  }
  const double pq = block_sum_parts(g.part + kPartPQ * kRedBlocks, g.np);
  const T al = (T)(S->rz[(it - 1) & 1] / pq);
  const T th = T(1.0 / kChebTheta);
  auto st = [&](int i, int, int, int) {
    UpdSt<T> u;
    u.r = rold[i] - al * q[i];
    u.dv = L.dinv[i];
    u.x1 = u.dv * u.r * th;
    return u;
  };
  auto val = [](const UpdSt<T>& u) { return u.x1; };
  T acc = T(0);
  auto emit = [&](int lin, int, const UpdSt<T>& u, T Ax) {
    const T xo = (it == 1) ? T(0) : __builtin_nontemporal_load(&x[lin]);
    __builtin_nontemporal_store(xo + al * __builtin_nontemporal_load(&p[lin]), &x[lin]);
    __builtin_nontemporal_store(u.r, &rnew[lin]);
    acc += u.r * u.r;
    xm[lin] = (T(1.0) + T(kChebC1)) * u.x1 + T(kChebC2) * u.dv * (u.r - Ax);
  };
  zmarch<T>(L, zchunk(L.n, zc), st, val, emit);
  block_partial((double)acc, g.part + kPartRR * kRedBlocks);
}

// k_cg_apply<T, 3> in z-marching form
template <class T>
__global__ void __launch_bounds__(kBlock) k_cg_apply_zm(LV<T> L, const T* z, const T* pold, T* pnew, T* q, T* x,
                                                        CGArgs g, int it, int zc) {
  CGCtl* S = g.ctl;
  if (S->flag) return;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  const double rz = block_sum_parts(g.part + kPartRZ * kRedBlocks, g.np);
  double beta = 0.0;
  if (it == 1) {
    const double bb = block_sum_parts(g.part + kPartBB * kRedBlocks, g.np);
    if (lead) S->bb = bb;
    if (bb == 0.0) {  // the update kernel of this iteration ends the solve
      FOR_CELLS(lin, L.N) x[lin] = T(0);
      return;
    }
  } else {
    beta = rz / S->rz[it & 1];
  }
  if (lead) S->rz[(it - 1) & 1] = rz;
  const T bt = (T)beta;
  const T* po = (it == 1) ? z : pold;
  auto st = [&](int i, int, int, int) { return z[i] + bt * po[i]; };
  auto val = [](T v) { return v; };
  T acc = T(0);
  auto emit = [&](int lin, int, T pc, T qv) {
    __builtin_nontemporal_store(pc, &pnew[lin]);
    __builtin_nontemporal_store(qv, &q[lin]);
    acc += pc * qv;
  };
  zmarch<T>(L, zchunk(L.n, zc), st, val, emit);
  block_partial((double)acc, g.part + kPartPQ * kRedBlocks);
}

template <class T>
struct PreSt {
  T b, dv, x1;  // right-hand side, inverse diagonal, first smoothing iterate
};

// k_mg_presmooth<T, 3, INIT> in z-marching form
template <class T, bool INIT>
__global__ void __launch_bounds__(kBlock) k_mg_presmooth_zm(LV<T> L, const T* b, T* x, CGArgs g, int zc) {
  if (INIT) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      g.ctl->flag = 0;
      g.ctl->its = 0;
    }
  } else if (g.ctl->flag) {
    return;
  }
  const T th = T(1.0 / kChebTheta);
  auto st = [&](int i, int, int, int) {
    PreSt<T> u;
    u.b = b[i];
    u.dv = L.dinv[i];
    u.x1 = u.dv * u.b * th;
    return u;
  };
  auto val = [](const PreSt<T>& u) { return u.x1; };
  T acc = T(0);
  auto emit = [&](int lin, int, const PreSt<T>& u, T Ax) {
    x[lin] = (T(1.0) + T(kChebC1)) * u.x1 + T(kChebC2) * u.dv * (u.b - Ax);
    if (INIT) acc += u.b * u.b;
  };
  zmarch<T>(L, zchunk(L.n, zc), st, val, emit);
  if (INIT) block_partial((double)acc, g.part + kPartBB * kRedBlocks);
}

// k_mg_smooth2<T, 3, RZ> in z-marching form
template <class T, bool RZ>
__global__ void __launch_bounds__(kBlock) k_mg_smooth2_zm(LV<T> L, const T* b, const T* x1, const T* d0, T* x,
                                                          CGArgs g, int zc) {
  if (g.ctl->flag) return;
  auto st = [&](int i, int, int, int) { return x1[i]; };
  auto val = [](T v) { return v; };
  T acc = T(0);
  auto emit = [&](int lin, int, T x1c, T Ax) {
    const T bl = __builtin_nontemporal_load(&b[lin]);
    const T r1 = bl - Ax;
    const T xn = x1c + T(kChebC1) * __builtin_nontemporal_load(&d0[lin]) + T(kChebC2) * __builtin_nontemporal_load(&L.dinv[lin]) * r1;
    __builtin_nontemporal_store(xn, &x[lin]);
    if (RZ) acc += bl * xn;
  };
  zmarch<T>(L, zchunk(L.n, zc), st, val, emit);
  if (RZ) block_partial((double)acc, g.part + kPartRZ * kRedBlocks);
}

// k_mg_prolong_smooth1<T, 3> in z-marching form
template <class T>
__global__ void __launch_bounds__(kBlock) k_mg_prolong_smooth1_zm(LV<T> L, const T* b, const T* x2, const T* xc,
                                                                  int cs0, int cs1, int cs2, T* x1, T* d0,
                                                                  CGArgs g, int zc) {
  if (g.ctl->flag) return;
  auto st = [&](int i, int cx, int cy, int cz) {
    return x2[i] + xc[(cx >> 1) * cs0 + (cy >> 1) * cs1 + (cz >> 1) * cs2];
  };
  auto val = [](T v) { return v; };
  auto emit = [&](int lin, int, T xpc, T Ax) {
    const T r0 = __builtin_nontemporal_load(&b[lin]) - Ax;
    const T dd = __builtin_nontemporal_load(&L.dinv[lin]) * r0 * T(1.0 / kChebTheta);
    x1[lin] = xpc + dd;
    __builtin_nontemporal_store(dd, &d0[lin]);
  };
  zmarch<T>(L, zchunk(L.n, zc), st, val, emit);
}

// k_mg_restrict_resid<T, 3, CONV> in z-marching form: a thread owns one coarse column and
// walks a chunk of coarse planes; the fine iterate of the plane below the current pair and
// of the pair itself, and the z face weights of the pair, are carried from one coarse plane
// to the next (the fine dimensions are even).  Each child's row is evaluated in apply_nb's
// order and the children are summed in restrict_at's order.
template <class T, bool CONV>
__global__ void __launch_bounds__(kBlock) k_mg_restrict_resid_zm(LV<T> L, const T* b, const T* x, T* bc,
                                                                 int ncx, int ncy, int ncz, int zc, CGArgs g,
                                                                 int it) {
  if (g.ctl->flag) return;
  if (CONV && blockIdx.x == 0) {
    const double rr = block_sum_parts(g.part + kPartRR * kRedBlocks, g.np);
    if (threadIdx.x == 0) cg_decide(g, rr, it);
  }
  const int nbx = (ncx + kZX - 1) / kZX, nby = (ncy + kZY - 1) / kZY;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int tile = blk % (nbx * nby), chunk = blk / (nbx * nby);
  const int ccx = (tile % nbx) * kZX + (int)threadIdx.x % kZX;
  const int ccy = (tile / nbx) * kZY + (int)threadIdx.x / kZX;
  const int cz0 = chunk * zc, cz1 = min(cz0 + zc, ncz);
  if (ccx >= ncx || ccy >= ncy || cz0 >= cz1) return;
  const int nz = L.n[2], sz = L.stride[2];
  // the four fine columns (child bits x, y) and their x/y coordinates
  int col[4], fx[4], fy[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    fx[q] = 2 * ccx + (q & 1);
    fy[q] = 2 * ccy + (q >> 1);
    col[q] = fx[q] + fy[q] * L.stride[1];
  }
  // x/y part of a fine row, in apply_nb's order, started from diag * xc
  auto rowxy = [&](int fl, int q, T xc) {
    T out = L.diag[fl] * xc;
    const int c2[2] = {fx[q], fy[q]};
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int n = L.n[d], st = L.stride[d];
      const int cm = (c2[d] == 0) ? fl + (n - 1) * st : fl - st;
      const int cp = (c2[d] == n - 1) ? fl - (n - 1) * st : fl + st;
      const T wl = L.w[d][fl];
      const T wu = (L.bc[d] == 1 && c2[d] == n - 1) ? T(0) : L.w[d][cp];
      out -= wu * (x[cp] - xc) - wl * (xc - x[cm]);
    }
    return out;
  };
  const int f00 = 2 * cz0;
  const int fm0 = (f00 == 0) ? nz - 1 : f00 - 1;
  T xA[4], xB[4], wB[4];  // x on the fine plane below the pair, x and w2 on its first plane
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    xA[q] = x[col[q] + fm0 * sz];
    xB[q] = x[col[q] + f00 * sz];
    wB[q] = L.w[2][col[q] + f00 * sz];
  }
  for (int cz = cz0; cz < cz1; ++cz) {
    const int f0 = 2 * cz, f1 = f0 + 1;
    const int f2 = (f1 == nz - 1) ? 0 : f1 + 1;
    T xC[4], xD[4], wC[4], wD[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      xC[q] = x[col[q] + f1 * sz];
      xD[q] = x[col[q] + f2 * sz];
      wC[q] = L.w[2][col[q] + f1 * sz];
      wD[q] = L.w[2][col[q] + f2 * sz];
    }
    T sum = T(0);
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) {
      const int q = ch & 3, k = ch >> 2;
      const int fl = col[q] + (k ? f1 : f0) * sz;
      const T xc = k ? xC[q] : xB[q];
      T out = rowxy(fl, q, xc);
      const T zp = k ? xD[q] : xC[q], zm = k ? xB[q] : xA[q];
      const T wl = k ? wC[q] : wB[q];
      const T wu = k ? ((L.bc[2] == 1 && f1 == nz - 1) ? T(0) : wD[q]) : wC[q];
      out -= wu * (zp - xc) - wl * (xc - zm);
      sum += __builtin_nontemporal_load(&b[fl]) - out;
    }
    bc[ccx + ccy * ncx + cz * ncx * ncy] = sum * T(1.0 / 8);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      xA[q] = xC[q];
      xB[q] = xD[q];
      wB[q] = wD[q];
    }
  }
}

// planes per chunk of the z-marching forms on level L, or 0 when its columns outnumber the
// partials (the grid-stride forms are used then)
static int zm_chunk(const Level& L) {
  const int nbx = (L.n[0] + kZX - 1) / kZX, nby = (L.n[1] + kZY - 1) / kZY;
  const int per = cg_partials((size_t)L.N) / (nbx * nby);
  if (per < 1) return 0;
  return (L.n[2] + per - 1) / per;
}

// ---- fused level pairs on LDS tiles ----------------------------------------------------
// One workgroup owns a tile of kBlock cells (16 x 16 in 2D, 8 x 8 x 4 in 3D) of the level it
// writes; the intermediate coarse vector lives in LDS with a halo of one cell, recomputed by
// every tile that needs it.
template <int ND>
struct TileDims;
template <>
struct TileDims<2> {
  static constexpr int X = 16, Y = 16, Z = 1;
};
template <>
struct TileDims<3> {
  static constexpr int X = 8, Y = 8, Z = 4;
};

__device__ __forceinline__ int wrapc(int c, int n) {
  c %= n;
  return c < 0 ? c + n : c;
}

template <int ND>
__device__ __forceinline__ void tile_origin(const int* n, int* o) {
  using TD = TileDims<ND>;
  const int nbx = (n[0] + TD::X - 1) / TD::X, nby = (n[1] + TD::Y - 1) / TD::Y;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  o[0] = (b % nbx) * TD::X;
  const int r = b / nbx;
  o[1] = (r % nby) * TD::Y;
  o[2] = (ND == 3) ? (r / nby) * TD::Z : 0;
}

template <int ND>
static int tile_blocks(const int* n) {
  using TD = TileDims<ND>;
  int b = ((n[0] + TD::X - 1) / TD::X) * ((n[1] + TD::Y - 1) / TD::Y);
  if (ND == 3) b *= (n[2] + TD::Z - 1) / TD::Z;
  return b;
}

// restriction of level F into level C (on C's tile and its halo, in LDS), then the first
// smoothing of level C on the tile.  CONV: block 0 also takes the convergence decision of
// iteration it (as k_mg_restrict_resid).
template <class T, int ND, bool CONV>
__global__ void __launch_bounds__(kBlock) k_mg_down(LV<T> F, const T* bf, const T* xf, LV<T> C, T* bc, T* xc,
                                                    CGArgs g, int it) {
  using TD = TileDims<ND>;
  constexpr int HX = TD::X + 2, HY = TD::Y + 2, HZ = (ND == 3) ? TD::Z + 2 : 1;
  constexpr int HN = HX * HY * HZ;
  __shared__ T sb[HN];
  if (g.ctl->flag) return;
  if (CONV && blockIdx.x == 0) {
    const double rr = block_sum_parts(g.part + kPartRR * kRedBlocks, g.np);
    if (threadIdx.x == 0) cg_decide(g, rr, it);
  }
  int o[3];
  tile_origin<ND>(C.n, o);
  const int t = threadIdx.x;
  const int l[3] = {t % TD::X, (t / TD::X) % TD::Y, t / (TD::X * TD::Y)};
  int c[3] = {o[0] + l[0], o[1] + l[1], (ND == 3) ? o[2] + l[2] : 0};
  const bool own = c[0] < C.n[0] && c[1] < C.n[1] && (ND < 3 || c[2] < C.n[2]);
  const int lin = own ? c[0] * C.stride[0] + c[1] * C.stride[1] + c[2] * C.stride[2] : 0;
  // the coarse row and the smoother's diagonal around it, ahead of the restriction phase
  RowCoef<T, ND> rc{};
  T dv = T(0), dvm[3] = {T(0), T(0), T(0)}, dvp[3] = {T(0), T(0), T(0)};
  if (own) {
    rc = row_coef<T, ND>(C, c, lin);
    dv = C.dinv[lin];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      dvm[d] = C.dinv[rc.cm[d]];
      dvp[d] = C.dinv[rc.cp[d]];
    }
  }
  for (int h = threadIdx.x; h < HN; h += kBlock) {
    const int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
    int cc[3] = {wrapc(o[0] + hx - 1, C.n[0]), wrapc(o[1] + hy - 1, C.n[1]),
                 (ND == 3) ? wrapc(o[2] + hz - 1, C.n[2]) : 0};
    sb[h] = restrict_at<T, ND>(F, bf, xf, cc);
  }
  __syncthreads();
  if (!own) return;
  const int hs[3] = {1, HX, HX * HY};
  const int hc = (l[0] + 1) + (l[1] + 1) * HX + ((ND == 3) ? (l[2] + 1) * HX * HY : 0);
  const T bcen = sb[hc];
  bc[lin] = bcen;
  const T th = T(1.0 / kChebTheta);
  auto x1 = [&](int d, int s, int) { return (s < 0 ? dvm[d] : dvp[d]) * sb[hc + s * hs[d]] * th; };
  const T x1c = dv * bcen * th;
  const T Ax = apply_row<T, ND>(rc, x1, x1c);
  xc[lin] = (T(1.0) + T(kChebC1)) * x1c + T(kChebC2) * dv * (bcen - Ax);
}

// second smoothing step of level C on the parents of F's tile and their halo (in LDS), then
// the prolongation to level F and its first post-smoothing step (as k_mg_prolong_smooth1).
template <class T, int ND>
__global__ void __launch_bounds__(kBlock) k_mg_up(LV<T> C, const T* bc, const T* t1c, const T* t2c, LV<T> F,
                                                  const T* bf, const T* x2f, T* t1f, T* t2f, CGArgs g) {
  using TD = TileDims<ND>;
  constexpr int PX = TD::X / 2 + 2, PY = TD::Y / 2 + 2, PZ = (ND == 3) ? TD::Z / 2 + 2 : 1;
  constexpr int PN = PX * PY * PZ;
  __shared__ T sx[PN];
  if (g.ctl->flag) return;
  int o[3];
  tile_origin<ND>(F.n, o);
  const int p0[3] = {o[0] / 2, o[1] / 2, o[2] / 2};
  const int t = threadIdx.x;
  const int l[3] = {t % TD::X, (t / TD::X) % TD::Y, t / (TD::X * TD::Y)};
  int c[3] = {o[0] + l[0], o[1] + l[1], (ND == 3) ? o[2] + l[2] : 0};
  const bool own = c[0] < F.n[0] && c[1] < F.n[1] && (ND < 3 || c[2] < F.n[2]);
  const int lin = own ? c[0] * F.stride[0] + c[1] * F.stride[1] + c[2] * F.stride[2] : 0;
  // the fine row, the fine iterate around it, b and the diagonal, ahead of the LDS phase
  RowCoef<T, ND> rf{};
  T x2c = T(0), x2m[3] = {T(0), T(0), T(0)}, x2p[3] = {T(0), T(0), T(0)}, bfc = T(0), dvf = T(0);
  if (own) {
    rf = row_coef<T, ND>(F, c, lin);
    x2c = x2f[lin];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      x2m[d] = x2f[rf.cm[d]];
      x2p[d] = x2f[rf.cp[d]];
    }
    bfc = bf[lin];
    dvf = F.dinv[lin];
  }
  auto t1 = [&](int k) { return t1c[k]; };
  for (int h = threadIdx.x; h < PN; h += kBlock) {
    const int hx = h % PX, hy = (h / PX) % PY, hz = h / (PX * PY);
    int cc[3] = {wrapc(p0[0] + hx - 1, C.n[0]), wrapc(p0[1] + hy - 1, C.n[1]),
                 (ND == 3) ? wrapc(p0[2] + hz - 1, C.n[2]) : 0};
    const int k = cc[0] * C.stride[0] + cc[1] * C.stride[1] + cc[2] * C.stride[2];
    const T x1c = t1c[k];
    const T r1 = bc[k] - apply_at<T, ND>(C, cc, k, t1, x1c);
    sx[h] = x1c + T(kChebC1) * t2c[k] + T(kChebC2) * C.dinv[k] * r1;
  }
  __syncthreads();
  if (!own) return;
  // LDS position of the parent of the fine cell f (unwrapped, at most one step from the tile)
  auto ppos = [&](const int* f) {
    int p = ((f[0] >> 1) - p0[0] + 1) + ((f[1] >> 1) - p0[1] + 1) * PX;
    if (ND == 3) p += ((f[2] >> 1) - p0[2] + 1) * PX * PY;
    return p;
  };
  const T xpc = x2c + sx[ppos(c)];
  auto xp = [&](int d, int s, int) {
    int f[3] = {c[0], c[1], c[2]};
    f[d] += s;
    return (s < 0 ? x2m[d] : x2p[d]) + sx[ppos(f)];
  };
  const T r0 = bfc - apply_row<T, ND>(rf, xp, xpc);
  const T dd = dvf * r0 * T(1.0 / kChebTheta);
  t1f[lin] = xpc + dd;
  t2f[lin] = dd;
}

// k_mg_up onto level 0 of a 2D grid followed by level 0's second post-smoothing with the
// (b, x) partials (k_mg_smooth2 with RZ): the first post-smoothing step is evaluated on the
// tile and on a ring of one cell around it (into LDS), the second on the tile from there.
// One block per tile, each writing one partial.  x2f is only read: the result goes to xo.
template <class T>
__global__ void __launch_bounds__(kBlock) k_mg_up_last(LV<T> C, const T* bc, const T* t1c, const T* t2c, LV<T> F,
                                                       const T* bf, const T* x2f, T* xo, CGArgs g) {
  using TD = TileDims<2>;
  constexpr int PX = TD::X / 2 + 2, PY = TD::Y / 2 + 2, PN = PX * PY;
  constexpr int QX = TD::X + 2, QY = TD::Y + 2, QN = QX * QY;
  __shared__ T sx[PN];
  __shared__ T s1[QN];
  __shared__ T s2[QN];
  if (g.ctl->flag) return;
  int o[3];
  tile_origin<2>(F.n, o);
  const int p0[2] = {o[0] / 2, o[1] / 2};
  // the coarse level's second smoothing on the parents of the tile and of two rings of cells
  // around it (as in k_mg_up)
  auto t1 = [&](int k) { return t1c[k]; };
  for (int h = threadIdx.x; h < PN; h += kBlock) {
    const int hx = h % PX, hy = h / PX;
    int cc[3] = {wrapc(p0[0] + hx - 1, C.n[0]), wrapc(p0[1] + hy - 1, C.n[1]), 0};
    const int k = cc[0] * C.stride[0] + cc[1] * C.stride[1];
    const T x1c = t1c[k];
    const T r1 = bc[k] - apply_at<T, 2>(C, cc, k, t1, x1c);
    sx[h] = x1c + T(kChebC1) * t2c[k] + T(kChebC2) * C.dinv[k] * r1;
  }
  __syncthreads();
  // LDS position of the parent of the fine cell with unwrapped coordinates (ux, uy)
  auto ppos = [&](int ux, int uy) { return ((ux >> 1) - p0[0] + 1) + ((uy >> 1) - p0[1] + 1) * PX; };
  // prolongation and the first post-smoothing step on the tile and its ring
  for (int h = threadIdx.x; h < QN; h += kBlock) {
    const int ux = o[0] + h % QX - 1, uy = o[1] + h / QX - 1;
    int fw[3] = {wrapc(ux, F.n[0]), wrapc(uy, F.n[1]), 0};
    const int lin = fw[0] * F.stride[0] + fw[1] * F.stride[1];
    const T xpc = x2f[lin] + sx[ppos(ux, uy)];
    auto xp = [&](int d, int sg, int k) {
      return x2f[k] + sx[d == 0 ? ppos(ux + sg, uy) : ppos(ux, uy + sg)];
    };
    const T r0 = bf[lin] - apply_nb<T, 2>(F, fw, lin, xp, xpc);
    const T dd = F.dinv[lin] * r0 * T(1.0 / kChebTheta);
    s1[h] = xpc + dd;
    s2[h] = dd;
  }
  __syncthreads();
  // the second post-smoothing step on the tile
  const int t = threadIdx.x;
  const int l[2] = {t % TD::X, t / TD::X};
  int c[3] = {o[0] + l[0], o[1] + l[1], 0};
  T acc = T(0);
  if (c[0] < F.n[0] && c[1] < F.n[1]) {
    const int lin = c[0] * F.stride[0] + c[1] * F.stride[1];
    const int hc = (l[0] + 1) + (l[1] + 1) * QX;
    const int hs[2] = {1, QX};
    const T x1c = s1[hc];
    auto xf = [&](int d, int sg, int) { return s1[hc + sg * hs[d]]; };
    const T r1 = bf[lin] - apply_nb<T, 2>(F, c, lin, xf, x1c);
    const T xn = x1c + T(kChebC1) * s2[hc] + T(kChebC2) * F.dinv[lin] * r1;
    xo[lin] = xn;
    acc += bf[lin] * xn;
  }
  block_partial((double)acc, g.part + kPartRZ * kRedBlocks);
}

#define CELLS(n) dim3(((n) + kBlock - 1) / kBlock), dim3(kBlock)

template <class T>
void launch_mg_down(const Grid& G, const Level& f, const T* bf, const T* xf, const Level& c, T* bc, T* xc,
                    const CGArgs& g, int conv_it, hipStream_t s) {
  LV<T> vf = view<T>(G, f), vc = view<T>(G, c);
  const double by = ((3.0 + G.nd) * f.N + (5.0 + G.nd) * c.N) * (double)sizeof(T);
  const int nb2 = tile_blocks<2>(c.n), nb3 = tile_blocks<3>(c.n);
  if (G.nd == 2) {
    if (conv_it > 0)
      launch_k(KF_MG_DOWN, by, k_mg_down<T, 2, true>, dim3(nb2), dim3(kBlock), 0, s, vf, bf, xf, vc, bc, xc, g,
               conv_it);
    else
      launch_k(KF_MG_DOWN, by, k_mg_down<T, 2, false>, dim3(nb2), dim3(kBlock), 0, s, vf, bf, xf, vc, bc, xc, g,
               0);
  } else {
    if (conv_it > 0)
      launch_k(KF_MG_DOWN, by, k_mg_down<T, 3, true>, dim3(nb3), dim3(kBlock), 0, s, vf, bf, xf, vc, bc, xc, g,
               conv_it);
    else
      launch_k(KF_MG_DOWN, by, k_mg_down<T, 3, false>, dim3(nb3), dim3(kBlock), 0, s, vf, bf, xf, vc, bc, xc, g,
               0);
  }
}
template <class T>
void launch_mg_up(const Grid& G, const Level& c, const T* bc, const T* t1c, const T* t2c, const Level& f,
                  const T* bf, const T* x2f, T* t1f, T* t2f, const CGArgs& g, hipStream_t s) {
  LV<T> vc = view<T>(G, c), vf = view<T>(G, f);
  const double by = ((5.0 + G.nd) * c.N + (6.0 + G.nd) * f.N) * (double)sizeof(T);
  if (G.nd == 2)
    launch_k(KF_MG_UP, by, k_mg_up<T, 2>, dim3(tile_blocks<2>(f.n)), dim3(kBlock), 0, s, vc, bc, t1c, t2c, vf, bf,
             x2f, t1f, t2f, g);
  else
    launch_k(KF_MG_UP, by, k_mg_up<T, 3>, dim3(tile_blocks<3>(f.n)), dim3(kBlock), 0, s, vc, bc, t1c, t2c, vf, bf,
             x2f, t1f, t2f, g);
}
template <class T>
bool launch_mg_up_last(const Grid& G, const Level& c, const T* bc, const T* t1c, const T* t2c, const Level& f,
                       const T* bf, const T* x2f, T* x, const CGArgs& g, hipStream_t s) {
  if (G.nd != 2) return false;
  const int nb = tile_blocks<2>(f.n);
  if (nb != g.np) return false;
  LV<T> vc = view<T>(G, c), vf = view<T>(G, f);
  const double by = ((5.0 + G.nd) * c.N + (5.0 + G.nd) * f.N) * (double)sizeof(T);
  launch_k(KF_MG_UP, by, k_mg_up_last<T>, dim3(nb), dim3(kBlock), 0, s, vc, bc, t1c, t2c, vf, bf, x2f, x, g);
  return true;
}


template <class T>
void launch_mg_presmooth(const Grid& G, const Level& L, const T* b, T* x, const CGArgs& g, bool init,
                         hipStream_t s) {
  LV<T> v = view<T>(G, L);
  const double by = (4.0 + G.nd) * L.N * (double)sizeof(T);
  if (G.nd == 3) {
    if (const int zc = zm_chunk(L)) {
      dim3 gr(red_grid(L.N)), bl(kBlock);
      if (init) launch_k(KF_MG_PRE, by, k_mg_presmooth_zm<T, true>, gr, bl, 0, s, v, b, x, g, zc);
      else launch_k(KF_MG_PRE, by, k_mg_presmooth_zm<T, false>, gr, bl, 0, s, v, b, x, g, zc);
      return;
    }
  }
  if (init) {
    dim3 gr(red_grid(L.N)), bl(kBlock);
    if (G.nd == 2) launch_k(KF_MG_PRE, by, k_mg_presmooth<T, 2, true>, gr, bl, 0, s, v, b, x, g);
    else launch_k(KF_MG_PRE, by, k_mg_presmooth<T, 3, true>, gr, bl, 0, s, v, b, x, g);
  } else {
    if (G.nd == 2) launch_k(KF_MG_PRE, by, k_mg_presmooth<T, 2, false>, CELLS(L.N), 0, s, v, b, x, g);
    else launch_k(KF_MG_PRE, by, k_mg_presmooth<T, 3, false>, CELLS(L.N), 0, s, v, b, x, g);
  }
}
template <class T>
void launch_mg_restrict_resid(const Grid& G, const Level& f, const T* b, const T* x, T* bc,
                              const Level& c, const CGArgs& g, int conv_it, hipStream_t s) {
  LV<T> v = view<T>(G, f);
  const double by = ((3.0 + G.nd) * f.N + c.N) * (double)sizeof(T);
  if (G.nd == 3) {
    const int nbx = (c.n[0] + kZX - 1) / kZX, nby = (c.n[1] + kZY - 1) / kZY;
    const int per = std::max(1, kRedBlocks / (nbx * nby));
    const int zc = (c.n[2] + per - 1) / per;
    const int nblk = nbx * nby * ((c.n[2] + zc - 1) / zc);
    if (conv_it > 0)
      launch_k(KF_MG_RESTRICT, by, k_mg_restrict_resid_zm<T, true>, dim3(nblk), dim3(kBlock), 0, s, v, b, x, bc,
               c.n[0], c.n[1], c.n[2], zc, g, conv_it);
    else
      launch_k(KF_MG_RESTRICT, by, k_mg_restrict_resid_zm<T, false>, dim3(nblk), dim3(kBlock), 0, s, v, b, x, bc,
               c.n[0], c.n[1], c.n[2], zc, g, 0);
    return;
  }
  if (conv_it > 0) {
    if (G.nd == 2)
      launch_k(KF_MG_RESTRICT, by, k_mg_restrict_resid<T, 2, true>, CELLS(c.N), 0, s, v, b, x, bc, c.N, c.n[0],
               c.n[1], g, conv_it);
    else
      launch_k(KF_MG_RESTRICT, by, k_mg_restrict_resid<T, 3, true>, CELLS(c.N), 0, s, v, b, x, bc, c.N, c.n[0],
               c.n[1], g, conv_it);
  } else {
    if (G.nd == 2)
      launch_k(KF_MG_RESTRICT, by, k_mg_restrict_resid<T, 2, false>, CELLS(c.N), 0, s, v, b, x, bc, c.N,
               c.n[0], c.n[1], g, 0);
    else
      launch_k(KF_MG_RESTRICT, by, k_mg_restrict_resid<T, 3, false>, CELLS(c.N), 0, s, v, b, x, bc, c.N,
               c.n[0], c.n[1], g, 0);
  }
}
template <class T>
void launch_mg_prolong_smooth1(const Grid& G, const Level& f, const T* b, const T* x2, const T* xc,
                               const Level& c, T* x1, T* d0, const CGArgs& g, hipStream_t s) {
  LV<T> v = view<T>(G, f);
  const double by = ((6.0 + G.nd) * f.N + c.N) * (double)sizeof(T);
  if (G.nd == 3) {
    if (const int zc = zm_chunk(f)) {
      launch_k(KF_MG_PROLONG, by, k_mg_prolong_smooth1_zm<T>, dim3(red_grid(f.N)), dim3(kBlock), 0, s, v, b, x2,
               xc, c.stride[0], c.stride[1], c.stride[2], x1, d0, g, zc);
      return;
    }
  }
  if (G.nd == 2)
    launch_k(KF_MG_PROLONG, by, k_mg_prolong_smooth1<T, 2>, CELLS(f.N), 0, s, v, b, x2, xc, c.stride[0],
             c.stride[1], c.stride[2], x1, d0, g);
  else
    launch_k(KF_MG_PROLONG, by, k_mg_prolong_smooth1<T, 3>, CELLS(f.N), 0, s, v, b, x2, xc, c.stride[0],
             c.stride[1], c.stride[2], x1, d0, g);
}
template <class T>
void launch_mg_smooth2(const Grid& G, const Level& L, const T* b, const T* x1, const T* d0, T* x,
                       const CGArgs& g, bool rz, hipStream_t s) {
  LV<T> v = view<T>(G, L);
  const double by = (6.0 + G.nd) * L.N * (double)sizeof(T);
  if (G.nd == 3) {
    if (const int zc = zm_chunk(L)) {
      dim3 gr(red_grid(L.N)), bl(kBlock);
      if (rz) launch_k(KF_MG_SMOOTH2, by, k_mg_smooth2_zm<T, true>, gr, bl, 0, s, v, b, x1, d0, x, g, zc);
      else launch_k(KF_MG_SMOOTH2, by, k_mg_smooth2_zm<T, false>, gr, bl, 0, s, v, b, x1, d0, x, g, zc);
      return;
    }
  }
  if (rz) {
    dim3 gr(red_grid(L.N)), bl(kBlock);
    if (G.nd == 2) launch_k(KF_MG_SMOOTH2, by, k_mg_smooth2<T, 2, true>, gr, bl, 0, s, v, b, x1, d0, x, g);
    else launch_k(KF_MG_SMOOTH2, by, k_mg_smooth2<T, 3, true>, gr, bl, 0, s, v, b, x1, d0, x, g);
  } else {
    if (G.nd == 2)
      launch_k(KF_MG_SMOOTH2, by, k_mg_smooth2<T, 2, false>, CELLS(L.N), 0, s, v, b, x1, d0, x, g);
    else
      launch_k(KF_MG_SMOOTH2, by, k_mg_smooth2<T, 3, false>, CELLS(L.N), 0, s, v, b, x1, d0, x, g);
  }
}

// ---- coarse part of the V-cycle in one workgroup -------------------------------------------
// Levels with at most kCoarseMaxN cells.  Right-hand sides, iterates and smoother vectors
// live in LDS, and so do the coefficients of every level for which the launch reserved room
// (coff >= 0; ALL_LDS: every level); phases are separated by barriers.  mode bits:
//   kCoarseInit     reset the control block, write the (b, b) partials of the first level;
//   kCoarseConv     take the convergence decision of iteration it first;
//   kCoarseRZ       write the (b, x) partials of the first level;
//   kCoarseFromPre  x0 already holds the first smoothing of the first level (skipped here);
//   kCoarseToUp     stop after the first post-smoothing step of the first level and write
//                   its (t1, t2) to t1_0, t2_0 instead of x0.
template <class T, int ND, bool ALL_LDS>
__global__ void __launch_bounds__(kCoarseThreads) k_vcycle_coarse(CoarseArgs a, CGArgs g, int mode, int it) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_stop;
  const int tid = threadIdx.x;
  const int NT = blockDim.x;
  if (mode & kCoarseInit) {
    if (tid == 0) {
      g.ctl->flag = 0;
      g.ctl->its = 0;
    }
  } else if (g.ctl->flag) {
    return;
  }
  if (mode & kCoarseConv) {
    const double rr = block_sum_parts(g.part + kPartRR * kRedBlocks, g.np);
    if (tid == 0) {
      cg_decide(g, rr, it);
      s_stop = g.ctl->flag;
    }
    __syncthreads();
    if (s_stop) return;
  }
  T* sb = (T*)smem_raw;
  T* sx = sb + a.tot;
  T* s1 = sx + a.tot;
  T* s2 = s1 + a.tot;
  T* sc = s2 + a.tot;
  const T th = T(1.0 / kChebTheta);
  for (int j = 0; j < a.nl; ++j) {
    if (!ALL_LDS && a.coff[j] < 0) continue;
    T* base = sc + a.coff[j];
    const int n = a.N[j];
    for (int i = tid; i < n; i += NT) {
      base[i] = ((const T*)a.diag[j])[i];
      base[n + i] = ((const T*)a.dinv[j])[i];
#pragma unroll
      for (int d = 0; d < ND; ++d) base[(2 + d) * n + i] = ((const T*)a.w[j][d])[i];
    }
  }
  T bbacc = T(0);
  for (int i = tid; i < a.N[0]; i += NT) {
    const T bi = ((const T*)a.b0)[i];
    sb[a.off[0] + i] = bi;
    bbacc += bi * bi;
    if (mode & kCoarseFromPre) sx[a.off[0] + i] = ((const T*)a.x0)[i];
  }
  if (mode & kCoarseInit) {
    block_partial((double)bbacc, g.part + kPartBB * kRedBlocks);
    for (int i = tid + 1; i < g.np; i += NT) g.part[kPartBB * kRedBlocks + i] = 0.0;
  }
  __syncthreads();
  auto level = [&](int j) {
    LV<T> L;
    for (int d = 0; d < 3; ++d) {
      L.n[d] = a.n[j][d];
      L.stride[d] = a.stride[j][d];
      L.bc[d] = a.bc[d];
    }
    L.N = a.N[j];
    if (ALL_LDS || a.coff[j] >= 0) {
      const T* base = sc + a.coff[j];
      L.diag = base;
      L.dinv = base + L.N;
      for (int d = 0; d < 3; ++d) L.w[d] = base + (2 + (d < ND ? d : 0)) * L.N;
    } else {
      L.diag = (const T*)a.diag[j];
      L.dinv = (const T*)a.dinv[j];
      for (int d = 0; d < 3; ++d) L.w[d] = (const T*)a.w[j][d];
    }
    return L;
  };
  for (int j = 0; j + 1 < a.nl; ++j) {
    const LV<T> L = level(j);
    const T* b = sb + a.off[j];
    T* x = sx + a.off[j];
    if (!(j == 0 && (mode & kCoarseFromPre))) {
      for (int i = tid; i < L.N; i += NT) {
        int c[3];
        coords<ND>(L.n, i, c);
        auto x1 = [&](int k) { return L.dinv[k] * b[k] * th; };
        T x1c = x1(i);
        T Ax = apply_at<T, ND>(L, c, i, x1, x1c);
        x[i] = (T(1.0) + T(kChebC1)) * x1c + T(kChebC2) * L.dinv[i] * (b[i] - Ax);
      }
      __syncthreads();
    }
    T* bc = sb + a.off[j + 1];
    const int Nc = a.N[j + 1];
    for (int ic = tid; ic < Nc; ic += NT) {
      int cc[3];
      coords<ND>(a.n[j + 1], ic, cc);
      // in 3D two children at a time: the full unroll spilled registers in this
      // 1024-thread kernel
      bc[ic] = restrict_at<T, ND, (ND == 3) ? 2 : (1 << ND)>(L, b, x, cc);
    }
    __syncthreads();
  }
  {
    const int j = a.nl - 1;
    const T* b = sb + a.off[j];
    T* x = sx + a.off[j];
    const int n = a.N[j];
    for (int i = tid; i < n; i += NT) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += a.Ainv[(size_t)i * n + k] * (double)b[k];
      x[i] = (T)s;
    }
    __syncthreads();
  }
  for (int j = a.nl - 2; j >= 0; --j) {
    const LV<T> L = level(j);
    const T* b = sb + a.off[j];
    T* x = sx + a.off[j];
    const T* xc = sx + a.off[j + 1];
    const bool to_up = (j == 0) && (mode & kCoarseToUp);
    T* t1 = s1 + a.off[j];
    T* t2 = s2 + a.off[j];
    const int cs[3] = {a.stride[j + 1][0], a.stride[j + 1][1], a.stride[j + 1][2]};
    for (int i = tid; i < L.N; i += NT) {
      int c[3];
      coords<ND>(L.n, i, c);
      auto xp = [&](int k) { return x[k] + xc[parent_of<T, ND>(L, k, cs)]; };
      T xpc = xp(i);
      T r0 = b[i] - apply_at<T, ND>(L, c, i, xp, xpc);
      T dd = L.dinv[i] * r0 * th;
      t1[i] = xpc + dd;
      t2[i] = dd;
      if (to_up) {
        ((T*)a.t1_0)[i] = xpc + dd;
        ((T*)a.t2_0)[i] = dd;
      }
    }
    if (to_up) return;
    __syncthreads();
    for (int i = tid; i < L.N; i += NT) {
      int c[3];
      coords<ND>(L.n, i, c);
      auto xf = [&](int k) { return t1[k]; };
      T x1c = t1[i];
      T r1 = b[i] - apply_at<T, ND>(L, c, i, xf, x1c);
      x[i] = x1c + T(kChebC1) * t2[i] + T(kChebC2) * L.dinv[i] * r1;
    }
    __syncthreads();
  }
  T rzacc = T(0);
  for (int i = tid; i < a.N[0]; i += NT) {
    const T xi = sx[a.off[0] + i];
    ((T*)a.x0)[i] = xi;
    rzacc += sb[a.off[0] + i] * xi;
  }
  if (mode & kCoarseRZ) {
    block_partial((double)rzacc, g.part + kPartRZ * kRedBlocks);
    for (int i = tid + 1; i < g.np; i += NT) g.part[kPartRZ * kRedBlocks + i] = 0.0;
  }
}

static int max_lds_bytes() {
  static int v = -1;
  if (v < 0) {
    int dev = 0;
    int val = 65536;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&val, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      val = 65536;
    v = val;
  }
  return v;
}

template <class T, int ND, bool ALL_LDS>
static void coarse_lds_attr(size_t shm) {
  static size_t set = 0;
  if (shm > 65536 && shm > set) {
    (void)hipFuncSetAttribute((const void*)k_vcycle_coarse<T, ND, ALL_LDS>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    set = shm;
  }
}

template <class T, int ND, bool ALL_LDS>
static void launch_coarse_k(const CoarseArgs& a, const CGArgs& g, int mode, int it, size_t shm, double bytes,
                            hipStream_t s) {
  coarse_lds_attr<T, ND, ALL_LDS>(shm);
  launch_k(KF_MG_COARSE, bytes, k_vcycle_coarse<T, ND, ALL_LDS>, dim3(1), dim3(kCoarseThreads), (unsigned)shm, s,
           a, g, mode, it);
}

template <class T>
void launch_vcycle_coarse(const Grid& G, const Level* lv, int nl, const double* Ainv, const T* b0,
                          T* x0, const CGArgs& g, int mode, int it, hipStream_t s) {
  CoarseArgs a{};
  a.nl = nl;
  int tot = 0;
  for (int j = 0; j < nl; ++j) {
    for (int d = 0; d < 3; ++d) {
      a.n[j][d] = lv[j].n[d];
      a.stride[j][d] = lv[j].stride[d];
      a.w[j][d] = lv[j].w[d];
    }
    a.N[j] = lv[j].N;
    a.diag[j] = lv[j].diag;
    a.dinv[j] = lv[j].dinv;
    a.off[j] = tot;
    tot += lv[j].N;
  }
  for (int d = 0; d < 3; ++d) a.bc[d] = G.bc[d];
  a.tot = tot;
  a.Ainv = Ainv;
  a.b0 = b0;
  a.x0 = x0;
  a.t1_0 = lv[0].t1;
  a.t2_0 = lv[0].t2;
  // coefficients in LDS, coarsest levels first, while they fit
  size_t shm = 4 * (size_t)tot * sizeof(T);
  const size_t cap = (size_t)max_lds_bytes() - 1024;  // static LDS of the kernel
  int coef = 0;
  bool all = true;
  for (int j = nl - 1; j >= 0; --j) {
    const size_t need = (size_t)(2 + G.nd) * lv[j].N;
    if (shm + (coef + need) * sizeof(T) <= cap) {
      a.coff[j] = coef;
      coef += (int)need;
    } else {
      a.coff[j] = -1;
      all = false;
    }
  }
  shm += (size_t)coef * sizeof(T);
  double cbytes = 8.0 * (double)lv[nl - 1].N * lv[nl - 1].N + 2.0 * lv[0].N * (double)sizeof(T);
  for (int j = 0; j < nl; ++j) cbytes += (3.0 + G.nd) * lv[j].N * (double)sizeof(T);
  if (G.nd == 2) {
    if (all) launch_coarse_k<T, 2, true>(a, g, mode, it, shm, cbytes, s);
    else launch_coarse_k<T, 2, false>(a, g, mode, it, shm, cbytes, s);
  } else {
    if (all) launch_coarse_k<T, 3, true>(a, g, mode, it, shm, cbytes, s);
    else launch_coarse_k<T, 3, false>(a, g, mode, it, shm, cbytes, s);
  }
}

template <class T>
__global__ void k_dense_matvec(int n, const double* A, const T* x, T* y, CGArgs g) {
  if (g.ctl->flag) return;
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < n; ++j) s += A[(size_t)i * n + j] * (double)x[j];
  y[i] = (T)s;
}
template <class T>
void launch_dense_matvec(int n, const double* A, const T* x, T* y, const CGArgs& g, hipStream_t s) {
  k_dense_matvec<T><<<CELLS(n), 0, s>>>(n, A, x, y, g);
}

// ---- Chebyshev smoothing of any degree (every level, grid-stride) ------------------------
// The kernels above fuse the two steps of the degree-2 smoother with their neighbours; other
// degrees take one launch per step: from zero, d = x = D^-1 b / theta; then, from x,
// d = c1 d + c2 D^-1 (b - A x) and x + d, with c1 = rho_i rho_{i-1}, c2 = 2 rho_i / delta of
// the Chebyshev semi-iteration on [0.5, 2] (cheb_coefs).  d is updated in place (each cell
// reads and writes only its own entry); x is read at the neighbours, so xout != xin.
void cheb_coefs(int k, double* c1, double* c2) {
  const double theta = kChebTheta, delta = 2.0 - kChebTheta, sigma = theta / delta;
  double rho = 1.0 / sigma;
  for (int i = 1; i < k; ++i) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    c1[i] = rn * rho;
    c2[i] = 2.0 * rn / delta;
    rho = rn;
  }
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_cheb_zero(int n, const T* dinv, const T* b, T* x, T* d, CGArgs g) {
  if (g.ctl->flag) return;
  const T th = T(1.0 / kChebTheta);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const T dd = dinv[i] * b[i] * th;
    x[i] = dd;
    d[i] = dd;
  }
}
template <class T, int ND>
__global__ void __launch_bounds__(kBlock) k_cheb_step(LV<T> L, const T* b, const T* xin, T* xout, T* d, T c1, T c2,
                                                      CGArgs g) {
  if (g.ctl->flag) return;
  auto xf = [&](int i) { return xin[i]; };
  FOR_CELLS(lin, L.N) {
    int c[3];
    coords<ND>(L.n, lin, c);
    const T xc = xin[lin];
    const T r = b[lin] - apply_at<T, ND>(L, c, lin, xf, xc);
    const T dd = c1 * d[lin] + c2 * (L.dinv[lin] * r);
    d[lin] = dd;
    xout[lin] = xc + dd;
  }
}
template <class T>
void launch_cheb_zero(const Grid& G, const Level& L, const T* b, T* x, T* d, const CGArgs& g, hipStream_t s) {
  (void)G;
  launch_k(KF_MG_PRE, 4.0 * L.N * sizeof(T), k_cheb_zero<T>, CELLS(L.N), 0, s, L.N, (const T*)L.dinv, b, x, d, g);
}
template <class T>
void launch_cheb_step(const Grid& G, const Level& L, const T* b, const T* xin, T* xout, T* d, double c1, double c2,
                      const CGArgs& g, hipStream_t s) {
  LV<T> v = view<T>(G, L);
  const double by = (7.0 + G.nd) * L.N * (double)sizeof(T);
  if (G.nd == 2)
    launch_k(KF_MG_SMOOTH2, by, k_cheb_step<T, 2>, CELLS(L.N), 0, s, v, b, xin, xout, d, (T)c1, (T)c2, g);
  else
    launch_k(KF_MG_SMOOTH2, by, k_cheb_step<T, 3>, CELLS(L.N), 0, s, v, b, xin, xout, d, (T)c1, (T)c2, g);
}

// ---- CG kernels ------------------------------------------------------------------------
// iteration it (1-based).  apply: p = z + beta p_old with beta = (r,z)_{it-1}/(r,z)_{it-2}
// (p = z when it = 1), q = A p, partials of (p, q).  It also stores (r,z)_{it-1}, and at
// it = 1 stores ||b||^2 and writes x = 0 when b = 0 (the solve then ends with no iteration).
// The flag is only ever set by a kernel whose own blocks need no other output of it: blocks
// of that launch may read it before or after the write.
template <class T, int ND>
__global__ void __launch_bounds__(kBlock) k_cg_apply(LV<T> L, const T* z, const T* pold, T* pnew, T* q, T* x,
                                                     CGArgs g, int it) {
  CGCtl* S = g.ctl;
  if (S->flag) return;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  const double rz = block_sum_parts(g.part + kPartRZ * kRedBlocks, g.np);
  double beta = 0.0;
  if (it == 1) {
    const double bb = block_sum_parts(g.part + kPartBB * kRedBlocks, g.np);
    if (lead) S->bb = bb;
    if (bb == 0.0) {  // the update kernel of this iteration ends the solve
      FOR_CELLS(lin, L.N) x[lin] = T(0);
      return;
    }
  } else {
    beta = rz / S->rz[it & 1];
  }
  if (lead) S->rz[(it - 1) & 1] = rz;
  const T bt = (T)beta;
  const T* po = (it == 1) ? z : pold;
  auto pf = [&](int i) { return z[i] + bt * po[i]; };
  T acc = T(0);
  FOR_CELLS(lin, L.N) {
    int c[3];
    coords<ND>(L.n, lin, c);
    const T pc = pf(lin);
    const T qv = apply_at<T, ND>(L, c, lin, pf, pc);
    __builtin_nontemporal_store(pc, &pnew[lin]);
    __builtin_nontemporal_store(qv, &q[lin]);
    acc += pc * qv;
  }
  block_partial((double)acc, g.part + kPartPQ * kRedBlocks);
}

// update: alpha = (r,z)_{it-1} / (p,q); x += alpha p; r_new = r_old - alpha q, partials of
// (r_new, r_new); PRE: also the first smoothing of the next V-cycle on level 0, xm.
template <class T, int ND, bool PRE>
__global__ void __launch_bounds__(kBlock) k_cg_update(LV<T> L, const T* rold, const T* q, const T* p, T* x,
                                                      T* rnew, T* xm, CGArgs g, int it) {
  CGCtl* S = g.ctl;
  if (S->flag) return;
  if (it == 1 && S->bb == 0.0) {  // b = 0: x = 0 was written by the apply kernel
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      S->its = 0;
      S->flag = 1;
    }
    return;
  }
  const double pq = block_sum_parts(g.part + kPartPQ * kRedBlocks, g.np);
  const T al = (T)(S->rz[(it - 1) & 1] / pq);
  const T th = T(1.0 / kChebTheta);
  auto rf = [&](int i) { return rold[i] - al * q[i]; };
  T acc = T(0);
  FOR_CELLS(lin, L.N) {
    const T xo = (it == 1) ? T(0) : x[lin];
    x[lin] = xo + al * p[lin];
    const T rc = rf(lin);
    rnew[lin] = rc;
    acc += rc * rc;
    if (PRE) {
      int c[3];
      coords<ND>(L.n, lin, c);
      auto x1 = [&](int i) { return L.dinv[i] * rf(i) * th; };
      const T x1c = L.dinv[lin] * rc * th;
      const T Ax = apply_at<T, ND>(L, c, lin, x1, x1c);
      xm[lin] = (T(1.0) + T(kChebC1)) * x1c + T(kChebC2) * L.dinv[lin] * (rc - Ax);
    }
  }
  block_partial((double)acc, g.part + kPartRR * kRedBlocks);
}

// control reset and (b, b) partials; convergence decision alone; (r, z) partials alone
// (used when level 0 is the dense coarsest level)
template <class T>
__global__ void __launch_bounds__(kBlock) k_cg_init(int n, const T* b, CGArgs g) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    g.ctl->flag = 0;
    g.ctl->its = 0;
  }
  T acc = T(0);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) acc += b[i] * b[i];
  block_partial((double)acc, g.part + kPartBB * kRedBlocks);
}
__global__ void __launch_bounds__(kBlock) k_cg_decide(CGArgs g, int it) {
  if (g.ctl->flag) return;
  const double rr = block_sum_parts(g.part + kPartRR * kRedBlocks, g.np);
  if (threadIdx.x == 0) cg_decide(g, rr, it);
}
template <class T>
__global__ void __launch_bounds__(kBlock) k_cg_dot_rz(int n, const T* r, const T* z, CGArgs g) {
  if (g.ctl->flag) return;
  T acc = T(0);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) acc += r[i] * z[i];
  block_partial((double)acc, g.part + kPartRZ * kRedBlocks);
}

template <class T>
void launch_cg_apply(const Grid& G, const Level& L, const T* z, const T* pold, T* pnew, T* q, T* x,
                     const CGArgs& g, int it, hipStream_t s) {
  LV<T> v = view<T>(G, L);
  const double by = (5.0 + G.nd) * L.N * (double)sizeof(T);
  dim3 gr(red_grid(L.N)), bl(kBlock);
  if (G.nd == 2) launch_k(KF_CG_APPLY, by, k_cg_apply<T, 2>, gr, bl, 0, s, v, z, pold, pnew, q, x, g, it);
  else if (const int zc = zm_chunk(L))
    launch_k(KF_CG_APPLY, by, k_cg_apply_zm<T>, gr, bl, 0, s, v, z, pold, pnew, q, x, g, it, zc);
  else launch_k(KF_CG_APPLY, by, k_cg_apply<T, 3>, gr, bl, 0, s, v, z, pold, pnew, q, x, g, it);
}
template <class T>
void launch_cg_update(const Grid& G, const Level& L, const T* rold, const T* q, const T* p, T* x, T* rnew,
                      T* xm, const CGArgs& g, int it, hipStream_t s) {
  LV<T> v = view<T>(G, L);
  dim3 gr(red_grid(L.N)), bl(kBlock);
  if (xm) {
    const double by = (9.0 + G.nd) * L.N * (double)sizeof(T);
    if (G.nd == 2)
      launch_k(KF_CG_UPDATE, by, k_cg_update<T, 2, true>, gr, bl, 0, s, v, rold, q, p, x, rnew, xm, g, it);
    else if (const int zc = zm_chunk(L))
      launch_k(KF_CG_UPDATE, by, k_cg_update_zm<T>, gr, bl, 0, s, v, rold, q, p, x, rnew, xm, g, it, zc);
    else
      launch_k(KF_CG_UPDATE, by, k_cg_update<T, 3, true>, gr, bl, 0, s, v, rold, q, p, x, rnew, xm, g, it);
  } else {
    const double by = 6.0 * L.N * (double)sizeof(T);
    if (G.nd == 2)
      launch_k(KF_CG_UPDATE, by, k_cg_update<T, 2, false>, gr, bl, 0, s, v, rold, q, p, x, rnew, xm, g, it);
    else
      launch_k(KF_CG_UPDATE, by, k_cg_update<T, 3, false>, gr, bl, 0, s, v, rold, q, p, x, rnew, xm, g, it);
  }
}
template <class T>
void launch_cg_init(int n, const T* b, const CGArgs& g, hipStream_t s) {
  k_cg_init<T><<<red_grid(n), kBlock, 0, s>>>(n, b, g);
}
void launch_cg_decide(const CGArgs& g, int it, hipStream_t s) { k_cg_decide<<<1, kBlock, 0, s>>>(g, it); }
template <class T>
void launch_cg_dot_rz(int n, const T* r, const T* z, const CGArgs& g, hipStream_t s) {
  k_cg_dot_rz<T><<<red_grid(n), kBlock, 0, s>>>(n, r, z, g);
}

// double <-> float with scaling by 1/sqrt(*nrm2) (to float) or sqrt(*nrm2) (back); a zero
// right-hand side stays zero, a non-finite one stays non-finite
__global__ void k_cast_scale_f32(size_t n, const double* src, const double* nrm2, float* dst) {
  const double sc = (*nrm2 == 0.0) ? 0.0 : 1.0 / sqrt(*nrm2);
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
    dst[i] = (float)(src[i] * sc);
}
__global__ void k_uncast_scale_f64(size_t n, const float* src, const double* nrm2, double* dst) {
  const double sc = sqrt(*nrm2);
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
    dst[i] = (double)src[i] * sc;
}
void launch_cast_scale_f32(size_t n, const double* src, const double* nrm2, float* dst, hipStream_t s) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  k_cast_scale_f32<<<(unsigned)b, kBlock, 0, s>>>(n, src, nrm2, dst);
}
void launch_uncast_scale_f64(size_t n, const float* src, const double* nrm2, double* dst, hipStream_t s) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  k_uncast_scale_f64<<<(unsigned)b, kBlock, 0, s>>>(n, src, nrm2, dst);
}

// ---- transforms of the preconditioner -----------------------------------------------------
// residual r of the cell (r = L v when scaled); only rho and E rows are needed here
__device__ __forceinline__ void r_cell(const Grid& G, const double* X, const double* v, int scaled,
                                       int lin, double* rr, double* rE, double vsc = 0.0) {
  double vr = vread(v, lin, vsc), vE = vread(v, G.N + lin, vsc);
  if (scaled) {
    double rho = X[lin], e = X[G.N + lin];
    vr *= rho;
    vE *= rho * e;
  }
  *rr = vr;
  *rE = vE;
}

// F~_u on the low-d face of cell lf (lower cell lm): (r_m - u_d rbar_rho)/rho_f, r = L v when
// scaled
__device__ __forceinline__ double fu_face(const Grid& G, const double* X, const double* v, int scaled,
                                          double alpha1, int d, int lf, int lm, double vsc = 0.0) {
  const double rho = X[lf], rhom = X[lm];
  const double rf = 0.5 * (rhom + rho);
  const double ud = X[(2 + d) * G.N + lf];
  double rm = vread(v, (2 + d) * G.N + lf, vsc), r0m = vread(v, lm, vsc), r0c = vread(v, lf, vsc);
  if (scaled) {
    const double csf = 0.5 * (sound_speed_rt(G, rhom, X[G.N + lm]) + sound_speed_rt(G, rho, X[G.N + lf]));
    rm *= rf * fmax(fabs(ud), alpha1 * csf);
    r0m *= rhom;
    r0c *= rho;
  }
  return (rm - ud * (0.5 * (r0m + r0c))) / rf;
}

// rhs_p = F_p/(Gamma1 p); schur: minus dt div F~_u (wall faces carry no F~_u)
template <int ND>
__global__ void __launch_bounds__(kBlock) k_pbp_in(Grid G, const double* X, const double* v, int scaled,
                                                   double alpha1, double dt, int schur, double* rhs_p,
                                                   const double* vn2) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (lin >= G.N) return;
  const double vsc = inv_norm(vn2);
  double rho = X[lin], e = X[G.N + lin];
  double r0, rE;
  r_cell(G, X, v, scaled, lin, &r0, &rE, vsc);
  const Thermo th = thermo_rt(G, rho, e);
  const double dpdr = th.dpdr, dpde = th.dpde;
  double Fp = (dpdr - (e / rho) * dpde) * r0 + (dpde / rho) * rE;
  const double g1p = G.a_rad == 0.0 ? G.gamma * (G.gamma - 1.0) * rho * e : th.G1 * th.p;
  double rhs = Fp / g1p;
  if (schur) {
    Pos P = make_pos<ND>(G, lin);
    double div = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      double flo = 0.0, fhi = 0.0;
      if (!(G.bc[d] == 1 && P.c[d] == 0)) {
        double s;
        const int im = gidx<ND>(G, P, 0, shift(off0(), d, -1), &s);
        flo = fu_face(G, X, v, scaled, alpha1, d, lin, im, vsc);
      }
      const bool top = (P.c[d] == G.n[d] - 1);
      if (!(G.bc[d] == 1 && top)) {
        const int ip = top ? lin - (G.n[d] - 1) * G.stride[d] : lin + G.stride[d];
        fhi = fu_face(G, X, v, scaled, alpha1, d, ip, lin, vsc);
      }
      div += (fhi - flo) * G.idx[d];
    }
    rhs -= dt * div;
  }
  rhs_p[lin] = rhs;
}

__global__ void __launch_bounds__(kBlock) k_pbp_rhsT(Grid G, const double* X, const double* v, int scaled,
                                                     double dt, const double* dp, double* rhs_T, const double* vn2) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (lin >= G.N) return;
  const double vsc = inv_norm(vn2);
  double rho = X[lin], e = X[G.N + lin];
  double r0, rE;
  r_cell(G, X, v, scaled, lin, &r0, &rE, vsc);
  const Thermo th = thermo_rt(G, rho, e);
  const double dpdr = th.dpdr, dpde = th.dpde;
  double Fp = (dpdr - (e / rho) * dpde) * r0 + (dpde / rho) * rE;
  double Fe = (rE - e * r0) / rho;
  rhs_T[lin] = rho * Fe + (dp[lin] / dt - Fp) / th.G1;
}

template <int ND>
__global__ void __launch_bounds__(kBlock) k_pbp_out(Grid G, const double* X, const double* v, int scaled,
                                                    double alpha1, double dt, const double* dp,
                                                    const double* dT, double zs, double* z, double alpha2,
                                                    double* zpart, const double* vn2) {
  const double gm1 = G.gamma - 1.0;
  const double vsc = inv_norm(vn2);
  const bool rad = G.a_rad != 0.0;
  double acc = 0.0;  // zpart: sum over the block's cells of (z / R)^2 (R the unknown scaling, alpha2)
  FOR_CELLS(lin, G.N) {
    Pos P = make_pos<ND>(G, lin);
    // every load of the cell goes out first, as one batch (the wall test and the optional
    // terms below no longer gate any of them); the arithmetic is unchanged
    int im[ND];
    double rhom[ND], em[ND], vm_raw[ND], v0m_raw[ND], ud[ND], dpm[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      double s;
      im[d] = gidx<ND>(G, P, 0, shift(off0(), d, -1), &s);
      rhom[d] = X[im[d]];
      em[d] = X[G.N + im[d]];
      vm_raw[d] = v[(2 + d) * G.N + lin];
      v0m_raw[d] = v[im[d]];
      ud[d] = X[(2 + d) * G.N + lin];
      dpm[d] = dp[im[d]];
    }
    const double rho = X[lin], e = X[G.N + lin];
    const double v0_raw = v[lin], vE_raw = v[G.N + lin];
    const double dpc = dp[lin];
    const double dTc = dT ? dT[lin] : 0.0;
    auto vs = [&](double x) { return vsc != 0.0 ? mul_nc(x, vsc) : x; };
    double r0 = vs(v0_raw), rE = vs(vE_raw);  // r_cell
    if (scaled) {
      r0 *= rho;
      rE *= rho * e;
    }
    const Thermo th = thermo_rt(G, rho, e);
    const double dpdr = th.dpdr, dpde = th.dpde;
    double Fp = (dpdr - (e / rho) * dpde) * r0 + (dpde / rho) * rE;
    double Fe = (rE - e * r0) / rho;
    double de;
    if (dT) de = rad ? th.cv * dTc : dTc / gm1;  // de = c_v dT
    else de = dt * Fe + (dpc - dt * Fp) / (th.G1 * rho);
    const double z0 = zs * ((dpc - dpde * de) / dpdr), z1 = zs * de;
    z[lin] = z0;
    z[G.N + lin] = z1;
    if (zpart) {
      const double q0 = z0 / rho, q1 = z1 / e;
      acc += q0 * q0;
      acc += q1 * q1;
    }
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      double rf = 0.5 * (rhom[d] + rho);
      double vm = vs(vm_raw[d]);
      double rm = vm;
      double r0m = vs(v0m_raw[d]);
      double r0c = vs(v0_raw);
      double csf = 0.0;
      if (scaled || zpart) csf = 0.5 * (sound_speed_rt(G, rhom[d], em[d]) + sound_speed_rt(G, rho, e));
      if (scaled) {
        rm = vm * rf * fmax(fabs(ud[d]), alpha1 * csf);
        r0m *= rhom[d];
        r0c *= rho;
      }
      double rbar = 0.5 * (r0m + r0c);
      double Fu = (rm - ud[d] * rbar) / rf;
      double grad = (G.bc[d] == 1 && P.c[d] == 0) ? 0.0 : (dpc - dpm[d]) / (rf * G.dx[d]);
      const double zu = zs * (dt * (Fu - grad));
      z[(2 + d) * G.N + lin] = zu;
      if (zpart) {
        const double q = zu / fmax(fabs(ud[d]), alpha2 * csf);
        acc += q * q;
      }
    }
  }
  if (zpart) block_partial(acc, zpart);
}

void launch_pbp_in(const Grid& G, const double* X, const double* v, int scaled, double alpha1,
                   double dt, int schur, double* rhs_p, hipStream_t s, const double* vn2) {
  const double by = 8.0 * G.N * (schur ? 2.0 * (2 + G.nd) + 1 : 5.0);
  if (G.nd == 2)
    launch_k(KF_PBP_IN, by, k_pbp_in<2>, CELLS(G.N), 0, s, G, X, v, scaled, alpha1, dt, schur, rhs_p, vn2);
  else
    launch_k(KF_PBP_IN, by, k_pbp_in<3>, CELLS(G.N), 0, s, G, X, v, scaled, alpha1, dt, schur, rhs_p, vn2);
}
void launch_pbp_rhsT(const Grid& G, const double* X, const double* v, int scaled, double alpha1,
                     double dt, const double* dp, double* rhs_T, hipStream_t s, const double* vn2) {
  (void)alpha1;
  k_pbp_rhsT<<<CELLS(G.N), 0, s>>>(G, X, v, scaled, dt, dp, rhs_T, vn2);
}
void launch_pbp_out(const Grid& G, const double* X, const double* v, int scaled, double alpha1,
                    double dt, const double* dp, const double* dT, double zscale, double* z, hipStream_t s,
                    double alpha2, const RedWS* zn2_ws, double* zn2, const double* vn2) {
  const double by = 8.0 * G.N * (3.0 * (2 + G.nd) + 1 + (dT ? 1 : 0));
  double* part = zn2 ? zn2_ws->part : nullptr;
  // with the norm, one partial per block of a reduction-sized grid
  const dim3 gr = zn2 ? dim3(red_grid(G.N)) : dim3((G.N + kBlock - 1) / kBlock);
  if (G.nd == 2)
    launch_k(KF_PBP_OUT, by, k_pbp_out<2>, gr, dim3(kBlock), 0, s, G, X, v, scaled, alpha1, dt, dp, dT, zscale, z,
             alpha2, part, vn2);
  else
    launch_k(KF_PBP_OUT, by, k_pbp_out<3>, gr, dim3(kBlock), 0, s, G, X, v, scaled, alpha1, dt, dp, dT, zscale, z,
             alpha2, part, vn2);
  if (zn2) launch_finalize_sum(*zn2_ws, red_grid(G.N), 1, zn2, s);
}

// ---- explicit instantiations ---------------------------------------------------------------
#define INST(T)                                                                                          \
  template void launch_ell_coarsen<T>(const Grid&, const Level&, const Level&, hipStream_t);            \
  template void launch_ell_dinv<T>(const Grid&, const Level&, hipStream_t);                              \
  template void launch_mg_presmooth<T>(const Grid&, const Level&, const T*, T*, const CGArgs&, bool,     \
                                       hipStream_t);                                                     \
  template void launch_mg_restrict_resid<T>(const Grid&, const Level&, const T*, const T*, T*,         \
                                            const Level&, const CGArgs&, int, hipStream_t);              \
  template void launch_mg_prolong_smooth1<T>(const Grid&, const Level&, const T*, const T*,             \
                                             const T*, const Level&, T*, T*, const CGArgs&, hipStream_t);\
  template void launch_mg_smooth2<T>(const Grid&, const Level&, const T*, const T*, const T*, T*,       \
                                     const CGArgs&, bool, hipStream_t);                                  \
  template bool launch_mg_up_last<T>(const Grid&, const Level&, const T*, const T*, const T*,           \
                                     const Level&, const T*, const T*, T*, const CGArgs&, hipStream_t);  \
  template void launch_dense_matvec<T>(int, const double*, const T*, T*, const CGArgs&, hipStream_t);   \
  template void launch_vcycle_coarse<T>(const Grid&, const Level*, int, const double*, const T*, T*,     \
                                        const CGArgs&, int, int, hipStream_t);                           \
  template void launch_mg_down<T>(const Grid&, const Level&, const T*, const T*, const Level&, T*, T*,  \
                                  const CGArgs&, int, hipStream_t);                                      \
  template void launch_mg_up<T>(const Grid&, const Level&, const T*, const T*, const T*, const Level&, \
                                const T*, const T*, T*, T*, const CGArgs&, hipStream_t);                 \
  template void launch_cg_apply<T>(const Grid&, const Level&, const T*, const T*, T*, T*, T*,           \
                                   const CGArgs&, int, hipStream_t);                                     \
  template void launch_cg_update<T>(const Grid&, const Level&, const T*, const T*, const T*, T*, T*, T*,\
                                    const CGArgs&, int, hipStream_t);                                    \
  template void launch_cg_init<T>(int, const T*, const CGArgs&, hipStream_t);                           \
  template void launch_cg_dot_rz<T>(int, const T*, const T*, const CGArgs&, hipStream_t);              \
  template void launch_cheb_zero<T>(const Grid&, const Level&, const T*, T*, T*, const CGArgs&,         \
                                    hipStream_t);                                                       \
  template void launch_cheb_step<T>(const Grid&, const Level&, const T*, const T*, T*, T*, double,      \
                                    double, const CGArgs&, hipStream_t);
INST(float)
INST(double)

}  // namespace jfnk
