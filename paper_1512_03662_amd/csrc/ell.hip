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

// (A phi)[c] with phi given by a functor of the linear index; phic = phi(lin)
template <class T, int ND, class F>
__device__ __forceinline__ T apply_at(const LV<T>& L, const int* c, int lin, const F& phi, T phic) {
  T out = L.diag[lin] * phic;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const int n = L.n[d], st = L.stride[d];
    const int cm = (c[d] == 0) ? lin + (n - 1) * st : lin - st;
    const int cp = (c[d] == n - 1) ? lin - (n - 1) * st : lin + st;
    const T wl = L.w[d][lin];
    const T wu = (L.bc[d] == 1 && c[d] == n - 1) ? T(0) : L.w[d][cp];
    out -= wu * (phi(cp) - phic) - wl * (phic - phi(cm));
  }
  return out;
}

// ---- coefficients ------------------------------------------------------------------------
template <int ND>
__global__ void __launch_bounds__(kBlock) k_ell_coef(Grid G, const double* X, double dt, int op, double* diag,
                                                     double* w0, double* w1, double* w2) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (lin >= G.N) return;
  Pos P = make_pos<ND>(G, lin);
  const double gm1 = G.gamma - 1.0;
  const double rho = X[lin], e = X[G.N + lin];
  double* w[3] = {w0, w1, w2};
  if (op == 0) {
    diag[lin] = 1.0 / (G.gamma * gm1 * rho * e * dt);
  } else {
    diag[lin] = rho / (gm1 * dt);
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
      double Tm = gm1 * X[G.N + im], T0 = gm1 * e;
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

// ---- V-cycle pieces ------------------------------------------------------------------------
template <class T, int ND>
__global__ void __launch_bounds__(kBlock) k_mg_presmooth(LV<T> L, const T* b, T* x) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (lin >= L.N) return;
  int c[3];
  coords<ND>(L.n, lin, c);
  const T th = T(1.0 / kChebTheta);
  auto x1 = [&](int i) { return L.dinv[i] * b[i] * th; };
  T x1c = x1(lin);
  T Ax = apply_at<T, ND>(L, c, lin, x1, x1c);
  x[lin] = (T(1.0) + T(kChebC1)) * x1c + T(kChebC2) * L.dinv[lin] * (b[lin] - Ax);
}

template <class T, int ND>
__global__ void __launch_bounds__(kBlock) k_mg_restrict_resid(LV<T> L, const T* b, const T* x, T* bc,
                                                              int Nc, int nc0, int nc1) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (lin >= Nc) return;
  int cc[3];
  cc[0] = lin % nc0;
  int r = lin / nc0;
  cc[1] = r % nc1;
  cc[2] = r / nc1;
  auto xf = [&](int i) { return x[i]; };
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
                                                               int cs0, int cs1, int cs2, T* x1, T* d0) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (lin >= L.N) return;
  int c[3];
  coords<ND>(L.n, lin, c);
  const int cst[3] = {cs0, cs1, cs2};
  auto xp = [&](int i) { return x2[i] + xc[parent_of<T, ND>(L, i, cst)]; };
  T xpc = xp(lin);
  T r0 = b[lin] - apply_at<T, ND>(L, c, lin, xp, xpc);
  T dd = L.dinv[lin] * r0 * T(1.0 / kChebTheta);
  x1[lin] = xpc + dd;
  d0[lin] = dd;
}

template <class T, int ND>
__global__ void __launch_bounds__(kBlock) k_mg_smooth2(LV<T> L, const T* b, const T* x1, const T* d0, T* x) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (lin >= L.N) return;
  int c[3];
  coords<ND>(L.n, lin, c);
  auto xf = [&](int i) { return x1[i]; };
  T x1c = x1[lin];
  T r1 = b[lin] - apply_at<T, ND>(L, c, lin, xf, x1c);
  x[lin] = x1c + T(kChebC1) * d0[lin] + T(kChebC2) * L.dinv[lin] * r1;
}

#define CELLS(n) dim3(((n) + kBlock - 1) / kBlock), dim3(kBlock)

template <class T>
void launch_mg_presmooth(const Grid& G, const Level& L, const T* b, T* x, hipStream_t s) {
  LV<T> v = view<T>(G, L);
  const double by = (4.0 + G.nd) * L.N * (double)sizeof(T);
  if (G.nd == 2) launch_k(KF_MG_PRE, by, k_mg_presmooth<T, 2>, CELLS(L.N), 0, s, v, b, x);
  else launch_k(KF_MG_PRE, by, k_mg_presmooth<T, 3>, CELLS(L.N), 0, s, v, b, x);
}
template <class T>
void launch_mg_restrict_resid(const Grid& G, const Level& f, const T* b, const T* x, T* bc,
                              const Level& c, hipStream_t s) {
  LV<T> v = view<T>(G, f);
  const double by = ((3.0 + G.nd) * f.N + c.N) * (double)sizeof(T);
  if (G.nd == 2)
    launch_k(KF_MG_RESTRICT, by, k_mg_restrict_resid<T, 2>, CELLS(c.N), 0, s, v, b, x, bc, c.N, c.n[0], c.n[1]);
  else
    launch_k(KF_MG_RESTRICT, by, k_mg_restrict_resid<T, 3>, CELLS(c.N), 0, s, v, b, x, bc, c.N, c.n[0], c.n[1]);
}
template <class T>
void launch_mg_prolong_smooth1(const Grid& G, const Level& f, const T* b, const T* x2, const T* xc,
                               const Level& c, T* x1, T* d0, hipStream_t s) {
  LV<T> v = view<T>(G, f);
  const double by = ((6.0 + G.nd) * f.N + c.N) * (double)sizeof(T);
  if (G.nd == 2)
    launch_k(KF_MG_PROLONG, by, k_mg_prolong_smooth1<T, 2>, CELLS(f.N), 0, s, v, b, x2, xc, c.stride[0],
             c.stride[1], c.stride[2], x1, d0);
  else
    launch_k(KF_MG_PROLONG, by, k_mg_prolong_smooth1<T, 3>, CELLS(f.N), 0, s, v, b, x2, xc, c.stride[0],
             c.stride[1], c.stride[2], x1, d0);
}
template <class T>
void launch_mg_smooth2(const Grid& G, const Level& L, const T* b, const T* x1, const T* d0, T* x,
                       hipStream_t s) {
  LV<T> v = view<T>(G, L);
  const double by = (6.0 + G.nd) * L.N * (double)sizeof(T);
  if (G.nd == 2) launch_k(KF_MG_SMOOTH2, by, k_mg_smooth2<T, 2>, CELLS(L.N), 0, s, v, b, x1, d0, x);
  else launch_k(KF_MG_SMOOTH2, by, k_mg_smooth2<T, 3>, CELLS(L.N), 0, s, v, b, x1, d0, x);
}

// ---- coarse part of the V-cycle in one workgroup -------------------------------------------
// Levels with at most kCoarseMaxN cells: right-hand side, iterate and smoother vectors live
// in LDS, coefficients are read from global memory; phases are separated by barriers.
template <class T, int ND>
__global__ void __launch_bounds__(kCoarseThreads) k_vcycle_coarse(CoarseArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sb = (T*)smem_raw;
  T* sx = sb + a.tot;
  T* s1 = sx + a.tot;
  T* s2 = s1 + a.tot;
  const int tid = threadIdx.x;
  const int NT = blockDim.x;
  const T th = T(1.0 / kChebTheta);
  for (int i = tid; i < a.N[0]; i += NT) sb[a.off[0] + i] = ((const T*)a.b0)[i];
  __syncthreads();
  for (int j = 0; j + 1 < a.nl; ++j) {
    LV<T> L;
    for (int d = 0; d < 3; ++d) {
      L.n[d] = a.n[j][d];
      L.stride[d] = a.stride[j][d];
      L.bc[d] = a.bc[d];
      L.w[d] = (const T*)a.w[j][d];
    }
    L.N = a.N[j];
    L.diag = (const T*)a.diag[j];
    L.dinv = (const T*)a.dinv[j];
    const T* b = sb + a.off[j];
    T* x = sx + a.off[j];
    for (int i = tid; i < L.N; i += NT) {
      int c[3];
      coords<ND>(L.n, i, c);
      auto x1 = [&](int k) { return L.dinv[k] * b[k] * th; };
      T x1c = x1(i);
      T Ax = apply_at<T, ND>(L, c, i, x1, x1c);
      x[i] = (T(1.0) + T(kChebC1)) * x1c + T(kChebC2) * L.dinv[i] * (b[i] - Ax);
    }
    __syncthreads();
    T* bc = sb + a.off[j + 1];
    const int Nc = a.N[j + 1];
    for (int ic = tid; ic < Nc; ic += NT) {
      int cc[3];
      coords<ND>(a.n[j + 1], ic, cc);
      auto xf = [&](int k) { return x[k]; };
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
      bc[ic] = sum * T(1.0 / (1 << ND));
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
    LV<T> L;
    for (int d = 0; d < 3; ++d) {
      L.n[d] = a.n[j][d];
      L.stride[d] = a.stride[j][d];
      L.bc[d] = a.bc[d];
      L.w[d] = (const T*)a.w[j][d];
    }
    L.N = a.N[j];
    L.diag = (const T*)a.diag[j];
    L.dinv = (const T*)a.dinv[j];
    const T* b = sb + a.off[j];
    T* x = sx + a.off[j];
    const T* xc = sx + a.off[j + 1];
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
    }
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
  for (int i = tid; i < a.N[0]; i += NT) ((T*)a.x0)[i] = sx[a.off[0] + i];
}

template <class T>
void launch_vcycle_coarse(const Grid& G, const Level* lv, int nl, const double* Ainv, const T* b0,
                          T* x0, hipStream_t s) {
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
  size_t shm = 4 * (size_t)tot * sizeof(T);
  double cbytes = 8.0 * (double)lv[nl - 1].N * lv[nl - 1].N + 2.0 * lv[0].N * (double)sizeof(T);
  for (int j = 0; j < nl; ++j) cbytes += (3.0 + G.nd) * lv[j].N * (double)sizeof(T);
  if (G.nd == 2)
    launch_k(KF_MG_COARSE, cbytes, k_vcycle_coarse<T, 2>, dim3(1), dim3(kCoarseThreads), (unsigned)shm, s, a);
  else
    launch_k(KF_MG_COARSE, cbytes, k_vcycle_coarse<T, 3>, dim3(1), dim3(kCoarseThreads), (unsigned)shm, s, a);
}

template <class T>
__global__ void k_dense_matvec(int n, const double* A, const T* x, T* y) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < n; ++j) s += A[(size_t)i * n + j] * (double)x[j];
  y[i] = (T)s;
}
template <class T>
void launch_dense_matvec(int n, const double* A, const T* x, T* y, hipStream_t s) {
  k_dense_matvec<T><<<CELLS(n), 0, s>>>(n, A, x, y);
}

// ---- CG vector kernels --------------------------------------------------------------------
template <class Op>
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// single-value block partial (the finalize kernel sums the partials in block order)
__device__ __forceinline__ void finish_sum(double v, double* out, const RedWS& ws) {
  constexpr int NW = kBlock / 64;
  __shared__ double sm[NW];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  v = wave_sum<int>(v);
  if (lane == 0) sm[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = sm[0];
    for (int w = 1; w < NW; ++w) a += sm[w];
    ws.part[blockIdx.x] = a;
  }
  (void)out;
}

static inline int red_grid(size_t n) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > (size_t)kRedBlocks) b = kRedBlocks;
  return (int)(b < 1 ? 1 : b);
}

template <class T, int ND>
__global__ void __launch_bounds__(kBlock) k_ell_apply_dot(LV<T> L, const T* p, T* q, double* out, RedWS ws) {
  T acc = T(0);
  auto pf = [&](int i) { return p[i]; };
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < L.N; lin += gridDim.x * kBlock) {
    int c[3];
    coords<ND>(L.n, lin, c);
    T pc = p[lin];
    T qv = apply_at<T, ND>(L, c, lin, pf, pc);
    q[lin] = qv;
    acc += pc * qv;
  }
  finish_sum((double)acc, out, ws);
}
template <class T>
void launch_ell_apply_dot(const Grid& G, const Level& L, const T* p, T* q, double* out,
                          const RedWS& ws, hipStream_t s) {
  LV<T> v = view<T>(G, L);
  {
    const double by = (3.0 + G.nd) * L.N * (double)sizeof(T);
    dim3 gr(red_grid(L.N)), bl(kBlock);
    if (G.nd == 2) launch_k(KF_CG_APPLY, by, k_ell_apply_dot<T, 2>, gr, bl, 0, s, v, p, q, out, ws);
    else launch_k(KF_CG_APPLY, by, k_ell_apply_dot<T, 3>, gr, bl, 0, s, v, p, q, out, ws);
  }
  launch_finalize_sum(ws, red_grid(L.N), 1, out, s);
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_cg_update(size_t n, const double* sc, int inum, int iden, T* x,
                                                      const T* p, T* r, const T* q, double* rr, RedWS ws) {
  const T a = (T)(sc[inum] / sc[iden]);
  T acc = T(0);
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    x[i] += a * p[i];
    T ri = r[i] - a * q[i];
    r[i] = ri;
    acc += ri * ri;
  }
  finish_sum((double)acc, rr, ws);
}
template <class T>
void launch_cg_update(size_t n, const double* sc, int i_num, int i_den, T* x, const T* p, T* r,
                      const T* q, double* rr, const RedWS& ws, hipStream_t s) {
  {
    launch_k(KF_CG_UPDATE, 6.0 * n * (double)sizeof(T), k_cg_update<T>, dim3(red_grid(n)), dim3(kBlock),
             0, s, n, sc, i_num, i_den, x, p, r, q, rr, ws);
  }
  launch_finalize_sum(ws, red_grid(n), 1, rr, s);
}

template <class T>
__global__ void k_cg_pupdate(size_t n, const double* sc, int inum, int iden, const T* z, T* p) {
  const T bta = (T)(sc[inum] / sc[iden]);
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
    p[i] = z[i] + bta * p[i];
}
template <class T>
void launch_cg_pupdate(size_t n, const double* sc, int i_num, int i_den, const T* z, T* p,
                       hipStream_t s) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  launch_k(KF_CG_PUPDATE, 3.0 * n * (double)sizeof(T), k_cg_pupdate<T>, dim3((unsigned)b), dim3(kBlock), 0,
           s, n, sc, i_num, i_den, z, p);
}

__global__ void k_cast_scale_f32(size_t n, const double* src, const double* nrm2, float* dst) {
  const double sc = 1.0 / sqrt(*nrm2);
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
                                       int lin, double* rr, double* rE) {
  double vr = v[lin], vE = v[G.N + lin];
  if (scaled) {
    double rho = X[lin], e = X[G.N + lin];
    vr *= rho;
    vE *= rho * e;
  }
  *rr = vr;
  *rE = vE;
}

template <int ND>
__global__ void __launch_bounds__(kBlock) k_pbp_in(Grid G, const double* X, const double* v, int scaled,
                                                   double* rhs_p) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (lin >= G.N) return;
  const double gm1 = G.gamma - 1.0;
  double rho = X[lin], e = X[G.N + lin];
  double r0, rE;
  r_cell(G, X, v, scaled, lin, &r0, &rE);
  double dpdr = gm1 * e, dpde = gm1 * rho;
  double Fp = (dpdr - (e / rho) * dpde) * r0 + (dpde / rho) * rE;
  rhs_p[lin] = Fp / (G.gamma * gm1 * rho * e);
}

__global__ void __launch_bounds__(kBlock) k_pbp_rhsT(Grid G, const double* X, const double* v, int scaled,
                                                     double dt, const double* dp, double* rhs_T) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (lin >= G.N) return;
  const double gm1 = G.gamma - 1.0;
  double rho = X[lin], e = X[G.N + lin];
  double r0, rE;
  r_cell(G, X, v, scaled, lin, &r0, &rE);
  double dpdr = gm1 * e, dpde = gm1 * rho;
  double Fp = (dpdr - (e / rho) * dpde) * r0 + (dpde / rho) * rE;
  double Fe = (rE - e * r0) / rho;
  rhs_T[lin] = rho * Fe + (dp[lin] / dt - Fp) / G.gamma;
}

template <int ND>
__global__ void __launch_bounds__(kBlock) k_pbp_out(Grid G, const double* X, const double* v, int scaled,
                                                    double alpha1, double dt, const double* dp,
                                                    const double* dT, double* z) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (lin >= G.N) return;
  Pos P = make_pos<ND>(G, lin);
  const double gm1 = G.gamma - 1.0;
  const double k = G.gamma * gm1;
  double rho = X[lin], e = X[G.N + lin];
  double r0, rE;
  r_cell(G, X, v, scaled, lin, &r0, &rE);
  double dpdr = gm1 * e, dpde = gm1 * rho;
  double Fp = (dpdr - (e / rho) * dpde) * r0 + (dpde / rho) * rE;
  double Fe = (rE - e * r0) / rho;
  double dpc = dp[lin];
  double de;
  if (dT) de = dT[lin] / gm1;
  else de = dt * Fe + (dpc - dt * Fp) / (G.gamma * rho);
  z[lin] = (dpc - dpde * de) / dpdr;
  z[G.N + lin] = de;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    double s;
    int im = gidx<ND>(G, P, 0, shift(off0(), d, -1), &s);
    double rhom = X[im];
    double rf = 0.5 * (rhom + rho);
    double vm = v[(2 + d) * G.N + lin];
    double rm = vm;
    double r0m = v[im];
    double r0c = v[lin];
    double ud = X[(2 + d) * G.N + lin];
    if (scaled) {
      double csf = 0.5 * (sqrt(k * X[G.N + im]) + sqrt(k * e));
      rm = vm * rf * fmax(fabs(ud), alpha1 * csf);
      r0m *= rhom;
      r0c *= rho;
    }
    double rbar = 0.5 * (r0m + r0c);
    double Fu = (rm - ud * rbar) / rf;
    double grad = (G.bc[d] == 1 && P.c[d] == 0) ? 0.0 : (dpc - dp[im]) / (rf * G.dx[d]);
    z[(2 + d) * G.N + lin] = dt * (Fu - grad);
  }
}

void launch_pbp_in(const Grid& G, const double* X, const double* v, int scaled, double alpha1,
                   double dt, double* rhs_p, hipStream_t s) {
  (void)alpha1;
  (void)dt;
  if (G.nd == 2) launch_k(KF_PBP_IN, 40.0 * G.N, k_pbp_in<2>, CELLS(G.N), 0, s, G, X, v, scaled, rhs_p);
  else launch_k(KF_PBP_IN, 40.0 * G.N, k_pbp_in<3>, CELLS(G.N), 0, s, G, X, v, scaled, rhs_p);
}
void launch_pbp_rhsT(const Grid& G, const double* X, const double* v, int scaled, double alpha1,
                     double dt, const double* dp, double* rhs_T, hipStream_t s) {
  (void)alpha1;
  k_pbp_rhsT<<<CELLS(G.N), 0, s>>>(G, X, v, scaled, dt, dp, rhs_T);
}
void launch_pbp_out(const Grid& G, const double* X, const double* v, int scaled, double alpha1,
                    double dt, const double* dp, const double* dT, double* z, hipStream_t s) {
  const double by = 8.0 * G.N * (3.0 * (2 + G.nd) + 1 + (dT ? 1 : 0));
  if (G.nd == 2) launch_k(KF_PBP_OUT, by, k_pbp_out<2>, CELLS(G.N), 0, s, G, X, v, scaled, alpha1, dt, dp, dT, z);
  else launch_k(KF_PBP_OUT, by, k_pbp_out<3>, CELLS(G.N), 0, s, G, X, v, scaled, alpha1, dt, dp, dT, z);
}

// ---- explicit instantiations ---------------------------------------------------------------
#define INST(T)                                                                                      \
  template void launch_ell_coarsen<T>(const Grid&, const Level&, const Level&, hipStream_t);        \
  template void launch_ell_dinv<T>(const Grid&, const Level&, hipStream_t);                          \
  template void launch_mg_presmooth<T>(const Grid&, const Level&, const T*, T*, hipStream_t);       \
  template void launch_mg_restrict_resid<T>(const Grid&, const Level&, const T*, const T*, T*,     \
                                            const Level&, hipStream_t);                              \
  template void launch_mg_prolong_smooth1<T>(const Grid&, const Level&, const T*, const T*,         \
                                             const T*, const Level&, T*, T*, hipStream_t);           \
  template void launch_mg_smooth2<T>(const Grid&, const Level&, const T*, const T*, const T*, T*,   \
                                     hipStream_t);                                                   \
  template void launch_dense_matvec<T>(int, const double*, const T*, T*, hipStream_t);              \
  template void launch_vcycle_coarse<T>(const Grid&, const Level*, int, const double*, const T*, T*, \
                                        hipStream_t);                                                \
  template void launch_ell_apply_dot<T>(const Grid&, const Level&, const T*, T*, double*,           \
                                        const RedWS&, hipStream_t);                                  \
  template void launch_cg_update<T>(size_t, const double*, int, int, T*, const T*, T*, const T*,    \
                                    double*, const RedWS&, hipStream_t);                             \
  template void launch_cg_pupdate<T>(size_t, const double*, int, int, const T*, T*, hipStream_t);
INST(float)
INST(double)

}  // namespace jfnk
