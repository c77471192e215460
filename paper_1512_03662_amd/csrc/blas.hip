// Vector kernels of the Krylov solvers: deterministic reductions (64-lane wavefront
// shuffles, then LDS across the 4 waves of a block, then per-block partials summed in block
// order by a one-block finalize kernel), the fused Gram-Schmidt passes of the Arnoldi step
// (Sect. 4.1: GMRES), linear combinations and the scaled norms of eq. nr_terminate.
//
// Every reduction visits elements in a fixed order for a given grid, so results are
// bitwise reproducible run to run.
#include <array>
#include <utility>

#include "common.hpp"
#include "kernels.hpp"
#include "probe.hpp"

namespace jfnk {

struct OpSum {
  static __device__ __forceinline__ double f(double a, double b) { return a + b; }
  static constexpr double id = 0.0;
};
// max that propagates NaN (fmax would return the other operand), so that a NaN anywhere in
// a max-reduction reaches the host's finiteness checks
__device__ __forceinline__ double nanmax(double a, double b) {
  return (a != a) ? a : ((b != b) ? b : fmax(a, b));
}
struct OpMax {
  static __device__ __forceinline__ double f(double a, double b) { return nanmax(a, b); }
  static constexpr double id = -HUGE_VAL;
};

template <class Op>
__device__ __forceinline__ double wave_reduce(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = Op::f(v, __shfl_xor(v, off, 64));
  return v;
}

// Reduce K per-thread values over the block and store the block's partials; a one-block
// finalize kernel launched next sums the partials in block order (no cross-block fences).
template <class Op, int K>
__device__ __forceinline__ void block_finish(const double (&vals)[K], double* out, const RedWS& ws) {
  constexpr int NW = kBlock / 64;
  __shared__ double sm[NW][K];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double v = wave_reduce<Op>(vals[k]);
    if (lane == 0) sm[wid][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double acc = sm[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < NW; ++w) acc = Op::f(acc, sm[w][threadIdx.x]);
    ws.part[(size_t)blockIdx.x * K + threadIdx.x] = acc;
  }
  (void)out;
}

// Sum k of K over the nb partials, combined in block order by one block; the result is
// valid in thread 0.
template <class Op>
__device__ __forceinline__ double finalize_one(const double* part, int nb, int K, int k, double* sm) {
  constexpr int NW = kBlock / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double acc = Op::id;
  for (int b = threadIdx.x; b < nb; b += kBlock) acc = Op::f(acc, part[(size_t)b * K + k]);
  acc = wave_reduce<Op>(acc);
  __syncthreads();
  if (lane == 0) sm[wid] = acc;
  __syncthreads();
  double s = sm[0];
  for (int w = 1; w < NW; ++w) s = Op::f(s, sm[w]);
  return s;
}

// One block combines the nb partials of each of the K sums in block order.
template <class Op>
__global__ void __launch_bounds__(kBlock) k_finalize(const double* part, int nb, int K, double* out) {
  __shared__ double sm[kBlock / 64];
  for (int k = 0; k < K; ++k) {
    const double s = finalize_one<Op>(part, nb, K, k, sm);
    if (threadIdx.x == 0) out[k] = s;
  }
}

template <class Op>
static void finalize(const RedWS& ws, int nb, int K, double* out, hipStream_t s) {
  k_finalize<Op><<<1, kBlock, 0, s>>>(ws.part, nb, K, out);
}

void launch_finalize_sum(const RedWS& ws, int nb, int K, double* out, hipStream_t s) {
  finalize<OpSum>(ws, nb, K, out, s);
}

static inline int red_blocks(size_t n) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > (size_t)kRedBlocks) b = kRedBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

// ---- dot ---------------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(kBlock) k_dot(size_t n, const T* a, const T* b, double* out, RedWS ws) {
  T acc = T(0);
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
    acc += a[i] * b[i];
  double v[1] = {(double)acc};
  block_finish<OpSum, 1>(v, out, ws);
}

template <class T>
void launch_dot(size_t n, const T* a, const T* b, double* out, const RedWS& w, hipStream_t s) {
  {
    launch_k(KF_DOT, 2.0 * sizeof(T) * n, k_dot<T>, dim3(red_blocks(n)), dim3(kBlock), 0, s, n, a, b,
             out, w);
  }
  finalize<OpSum>(w, red_blocks(n), 1, out, s);
}
template void launch_dot<double>(size_t, const double*, const double*, double*, const RedWS&, hipStream_t);
template void launch_dot<float>(size_t, const float*, const float*, double*, const RedWS&, hipStream_t);

// ---- Gram-Schmidt with delayed reorthogonalisation (two passes per Arnoldi step) ----------
// Each pass streams the basis once: its loads and stores are non-temporal.
// Slots 0..K-2 of V hold the finished orthonormal basis, slot j = K-1 the newest vector q~
// after one orthogonalisation (normalised by that pass's norm), w the new product.
// Pass 1: a_i = V_i . q~ and b_i = V_i . w for i <= j (2K sums).
// qn2 (optional): slot K-1 is kept unnormalised and read as V_{K-1} / sqrt(*qn2)
// The K + 1 loads of an element are all issued before its first product (a scheduling
// barrier keeps them together): left to itself the compiler interleaves them with the
// products for some K, down to one load in flight per wave.
template <int K>
__global__ void __launch_bounds__(kBlock) k_dcgs2_dots(size_t n, const double* V, size_t ld, const double* w,
                                                       const double* qn2, RedWS ws) {
  double acc[2 * K];
#pragma unroll
  for (int k = 0; k < 2 * K; ++k) acc[k] = 0.0;
  const double qsc = inv_norm(qn2);
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    double v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = __builtin_nontemporal_load(&V[k * ld + i]);
    const double wi = __builtin_nontemporal_load(&w[i]);
    __builtin_amdgcn_sched_barrier(0);
    const double qi = qsc != 0.0 ? mul_nc(v[K - 1], qsc) : v[K - 1];
#pragma unroll
    for (int k = 0; k < K - 1; ++k) {
      acc[k] += v[k] * qi;
      acc[K + k] += v[k] * wi;
    }
    acc[K - 1] += qi * qi;
    acc[2 * K - 1] += qi * wi;
  }
  block_finish<OpSum, 2 * K>(acc, nullptr, ws);
}

// Coefficients of pass 2 from the sums of pass 1 (j = K - 1; j = 0: q~ is final already):
// s_i = a_i, nu = sqrt(a_j - sum s_i^2), h_i = b_i (i < j), h_j = (b_j - sum s_i b_i) / nu.
// The host forms the same numbers for the Hessenberg matrix.
template <int K>
__device__ __forceinline__ void dcgs2_coef(const double* sums, double* sc, double& inv_nu, double* h) {
  constexpr int j = K - 1;
  double ss = 0.0, sb = 0.0;
#pragma unroll
  for (int k = 0; k < j; ++k) {
    sc[k] = sums[k];
    h[k] = sums[K + k];
    ss += sc[k] * sc[k];
    sb += sc[k] * h[k];
  }
  const double nu = (j == 0) ? 1.0 : sqrt(sums[j] - ss);
  inv_nu = 1.0 / nu;
  h[j] = (sums[K + j] - sb) * inv_nu;
}

// Pass 2: q = (q~ - sum_{i<j} s_i V_i) / nu replaces slot j (j >= 1), dst = w - sum_{i<j} h_i V_i
// - h_j q, and the partial sums of ||dst||^2.
template <int K>
__global__ void __launch_bounds__(kBlock) k_dcgs2_update(size_t n, double* V, size_t ld, const double* sums,
                                                         const double* w, double* dst, const double* qn2,
                                                         RedWS ws) {
  constexpr int j = K - 1;
  double sc[K], h[K], inv_nu;
  dcgs2_coef<K>(sums, sc, inv_nu, h);
  const double qsc = inv_norm(qn2);
  double acc[1] = {0.0};
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    double v[K];  // every load of the element before the first product, as in k_dcgs2_dots
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = __builtin_nontemporal_load(&V[k * ld + i]);
    double wi = __builtin_nontemporal_load(&w[i]);
    __builtin_amdgcn_sched_barrier(0);
    double q = qsc != 0.0 ? mul_nc(v[j], qsc) : v[j];
#pragma unroll
    for (int k = 0; k < j; ++k) {
      q -= sc[k] * v[k];
      wi -= h[k] * v[k];
    }
    if (j > 0) {
      q *= inv_nu;
      __builtin_nontemporal_store(q, &V[j * ld + i]);
    }
    wi -= h[j] * q;
    __builtin_nontemporal_store(wi, &dst[i]);
    acc[0] += wi * wi;
  }
  block_finish<OpSum, 1>(acc, nullptr, ws);
}

template <int K>
__global__ void __launch_bounds__(kBlock) k_lincomb(size_t n, const double* Z, size_t ld, const double* y,
                                                    double* dst) {
  double yk[K];
#pragma unroll
  for (int k = 0; k < K; ++k) yk[k] = y[k];
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    double z[K];  // every load of the element before the first product, as in k_dcgs2_dots
#pragma unroll
    for (int k = 0; k < K; ++k) z[k] = Z[k * ld + i];
    __builtin_amdgcn_sched_barrier(0);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) s += yk[k] * z[k];
    dst[i] = s;
  }
}

using MdFn = void (*)(size_t, const double*, size_t, const double*, const double*, double*, double*,
                      const RedWS&, hipStream_t);

template <int K>
static void lc_launch(size_t n, const double* Z, size_t ld, const double* y, const double* w,
                      double* dst, double* out, const RedWS& ws, hipStream_t s) {
  (void)w;
  (void)out;
  (void)ws;
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > 4096) b = 4096;
  launch_k(KF_LINCOMB, 8.0 * n * (K + 1), k_lincomb<K>, dim3((unsigned)b), dim3(kBlock), 0, s, n, Z,
           ld, y, dst);
}

// the sums are finalised by 2K blocks, one per sum (each in block order, as finalize)
__global__ void __launch_bounds__(kBlock) k_finalize_each(const double* part, int nb, int K, double* out) {
  __shared__ double sm[kBlock / 64];
  const double v = finalize_one<OpSum>(part, nb, K, blockIdx.x, sm);
  if (threadIdx.x == 0) out[blockIdx.x] = v;
}

// the two Gram-Schmidt passes of one Arnoldi step (K = j + 1 slots), one table entry per K
using GsFn = void (*)(size_t n, double* V, size_t ld, const double* w, const double* sums, double* dst,
                      double* out, const double* qn2, const RedWS& ws, hipStream_t s);
template <int K>
static void d1_launch(size_t n, double* V, size_t ld, const double* w, const double*, double*, double* out,
                      const double* qn2, const RedWS& ws, hipStream_t s) {
  launch_k(KF_GS_DOTS, 8.0 * n * (K + 1), k_dcgs2_dots<K>, dim3(red_blocks(n)), dim3(kBlock), 0, s, n,
           (const double*)V, ld, w, qn2, ws);
  k_finalize_each<<<2 * K, kBlock, 0, s>>>(ws.part, red_blocks(n), 2 * K, out);
}
template <int K>
static void d2_launch(size_t n, double* V, size_t ld, const double* w, const double* sums, double* dst,
                      double* out, const double* qn2, const RedWS& ws, hipStream_t s) {
  // reads slots 0..j and w; writes slot j (j >= 1) and dst
  const double by = 8.0 * n * (K + 1 + (K > 1 ? 2 : 1));
  launch_k(KF_GS_UPDATE, by, k_dcgs2_update<K>, dim3(red_blocks(n)), dim3(kBlock), 0, s, n, V, ld, sums, w,
           dst, qn2, ws);
  finalize<OpSum>(ws, red_blocks(n), 1, out, s);
}

constexpr int kMaxBasis = kMaxK - 1;  // K ranges over 1..kMaxBasis

template <template <int> class F, size_t... I>
constexpr std::array<MdFn, sizeof...(I)> make_table(std::index_sequence<I...>) {
  return {{&F<(int)I + 1>::run...}};
}
template <int K> struct LcT { static void run(size_t n, const double* V, size_t ld, const double* h, const double* w, double* m, double* o, const RedWS& ws, hipStream_t s) { lc_launch<K>(n, V, ld, h, w, m, o, ws, s); } };

static const auto kLc = make_table<LcT>(std::make_index_sequence<kMaxBasis>{});
template <int K> struct D1T { static constexpr GsFn run = &d1_launch<K>; };
template <int K> struct D2T { static constexpr GsFn run = &d2_launch<K>; };
template <template <int> class F, size_t... I>
constexpr std::array<GsFn, sizeof...(I)> make_gs_table(std::index_sequence<I...>) {
  return {{F<(int)I + 1>::run...}};
}
static const auto kD1 = make_gs_table<D1T>(std::make_index_sequence<kMaxBasis - 1>{});
static const auto kD2 = make_gs_table<D2T>(std::make_index_sequence<kMaxBasis - 1>{});

void launch_dcgs2_dots(size_t n, const double* V, size_t ld, int K, const double* w, double* sums,
                       const RedWS& ws, hipStream_t s, const double* qn2) {
  kD1[K - 1](n, const_cast<double*>(V), ld, w, nullptr, nullptr, sums, qn2, ws, s);
}
void launch_dcgs2_update(size_t n, double* V, size_t ld, int K, const double* sums, const double* w, double* dst,
                         double* nrm2, const RedWS& ws, hipStream_t s, const double* qn2) {
  kD2[K - 1](n, V, ld, w, sums, dst, nrm2, qn2, ws, s);
}

void launch_lincomb(size_t n, const double* Z, size_t ld, int K, const double* y, double* dst,
                    hipStream_t s) {
  kLc[K - 1](n, Z, ld, y, nullptr, dst, nullptr, RedWS{}, s);
}

// ---- elementwise -------------------------------------------------------------------------
__global__ void k_scale_by_inv_sqrt(size_t n, const double* src, const double* nrm2, double* dst) {
  double sc = 1.0 / sqrt(*nrm2);
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
    dst[i] = src[i] * sc;
}
void launch_scale_by_inv_sqrt(size_t n, const double* src, const double* nrm2, double* dst,
                              hipStream_t s) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  k_scale_by_inv_sqrt<<<(unsigned)b, kBlock, 0, s>>>(n, src, nrm2, dst);
}

__global__ void k_axpy(size_t n, double a, const double* x, double* y) {
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
    y[i] += a * x[i];
}
void launch_axpy(size_t n, double a, const double* x, double* y, hipStream_t s) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  k_axpy<<<(unsigned)b, kBlock, 0, s>>>(n, a, x, y);
}

template <class T>
__global__ void k_fill(size_t n, T v, T* y) {
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
    y[i] = v;
}
void launch_fill(size_t n, double v, double* y, hipStream_t s) { launch_fill_t<double>(n, v, y, s); }
template <class T>
void launch_fill_t(size_t n, T v, T* y, hipStream_t s) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  k_fill<T><<<(unsigned)b, kBlock, 0, s>>>(n, v, y);
}
template void launch_fill_t<double>(size_t, double, double*, hipStream_t);
template void launch_fill_t<float>(size_t, float, float*, hipStream_t);

// ---- scaled norms (R of Sect. 4.1 recomputed from X) ------------------------------------
template <int ND, bool RAD>
__device__ __forceinline__ void cell_R_scale(const Grid& G, const Pos& P, const double* X, double alpha2,
                                             double* Rs) {
  double e0 = X[G.N + P.lin];
  double cs0 = sound_speed<RAD>(G, X[P.lin], e0);
  Rs[0] = X[P.lin];
  Rs[1] = e0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    double s;
    int im = gidx<ND>(G, P, 1, shift(off0(), d, -1), &s);
    double csf = 0.5 * (sound_speed<RAD>(G, X[im], X[G.N + im]) + cs0);
    Rs[2 + d] = fmax(fabs(X[(2 + d) * G.N + P.lin]), alpha2 * csf);
  }
}

template <int ND, bool MAX, bool RAD>
__global__ void __launch_bounds__(kBlock) k_scaled_red(Grid G, const double* X, const double* V,
                                                       double alpha2, double* out, RedWS ws) {
  double acc = 0.0;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < G.N; lin += gridDim.x * kBlock) {
    Pos P = make_pos<ND>(G, lin);
    double Rs[2 + ND];
    cell_R_scale<ND, RAD>(G, P, X, alpha2, Rs);
#pragma unroll
    for (int v = 0; v < 2 + ND; ++v) {
      double q = V[v * G.N + lin] / Rs[v];
      if (MAX) acc = nanmax(acc, fabs(q));
      else acc += q * q;
    }
  }
  double a[1] = {acc};
  if (MAX) block_finish<OpMax, 1>(a, out, ws);
  else block_finish<OpSum, 1>(a, out, ws);
}

void launch_scaled_norm2(const Grid& G, const double* X, const double* V, double alpha2,
                         double* out, const RedWS& ws, hipStream_t s) {
  int b = red_blocks(G.N);
  {
    const double by = 16.0 * (2 + G.nd) * G.N;
    const bool rad = G.a_rad != 0.0;
    if (G.nd == 2)
      launch_k(KF_SCALED, by, rad ? k_scaled_red<2, false, true> : k_scaled_red<2, false, false>, dim3(b),
               dim3(kBlock), 0, s, G, X, V, alpha2, out, ws);
    else
      launch_k(KF_SCALED, by, rad ? k_scaled_red<3, false, true> : k_scaled_red<3, false, false>, dim3(b),
               dim3(kBlock), 0, s, G, X, V, alpha2, out, ws);
  }
  finalize<OpSum>(ws, b, 1, out, s);
}
// out[0] = max |V / R(X)|, out[1] = max over cells of -min(rho, e) of X + sgn V: the Newton
// correction's size and whether the corrected state keeps rho > 0 and e > 0 (out[1] < 0)
template <int ND, bool RAD>
__global__ void __launch_bounds__(kBlock) k_newton_check(Grid G, const double* X, const double* V, double alpha2,
                                                         double sgn, double* out, RedWS ws) {
  double acc[2] = {0.0, -HUGE_VAL};
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < G.N; lin += gridDim.x * kBlock) {
    Pos P = make_pos<ND>(G, lin);
    double Rs[2 + ND];
    cell_R_scale<ND, RAD>(G, P, X, alpha2, Rs);
#pragma unroll
    for (int v = 0; v < 2 + ND; ++v) acc[0] = nanmax(acc[0], fabs(V[v * G.N + lin] / Rs[v]));
    const double r1 = X[lin] + sgn * V[lin], e1 = X[G.N + lin] + sgn * V[G.N + lin];
    acc[1] = nanmax(acc[1], nanmax(-r1, -e1));
  }
  block_finish<OpMax, 2>(acc, out, ws);
}
void launch_newton_check(const Grid& G, const double* X, const double* V, double alpha2, double sgn,
                         double* out, const RedWS& ws, hipStream_t s) {
  int b = red_blocks(G.N);
  const bool rad = G.a_rad != 0.0;
  if (G.nd == 2) {
    if (rad) k_newton_check<2, true><<<b, kBlock, 0, s>>>(G, X, V, alpha2, sgn, out, ws);
    else k_newton_check<2, false><<<b, kBlock, 0, s>>>(G, X, V, alpha2, sgn, out, ws);
  } else {
    if (rad) k_newton_check<3, true><<<b, kBlock, 0, s>>>(G, X, V, alpha2, sgn, out, ws);
    else k_newton_check<3, false><<<b, kBlock, 0, s>>>(G, X, V, alpha2, sgn, out, ws);
  }
  finalize<OpMax>(ws, b, 2, out, s);
}

// max_c (|u_c| + c_s), u_c the mean of the two faces of c along each axis (Introduction)
template <int ND>
__global__ void __launch_bounds__(kBlock) k_cfl_speed(Grid G, const double* X, double* out, RedWS ws) {
  double acc = 0.0;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < G.N; lin += gridDim.x * kBlock) {
    Pos P = make_pos<ND>(G, lin);
    double u2 = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      double s0, s1;
      int i0 = gidx<ND>(G, P, 2 + d, off0(), &s0);
      int i1 = gidx<ND>(G, P, 2 + d, shift(off0(), d, 1), &s1);
      double uc = 0.5 * (s0 * X[(2 + d) * G.N + i0] + s1 * X[(2 + d) * G.N + i1]);
      u2 += uc * uc;
    }
    acc = nanmax(acc, sqrt(u2) + sound_speed_rt(G, X[lin], X[G.N + lin]));
  }
  double a[1] = {acc};
  block_finish<OpMax, 1>(a, out, ws);
}
void launch_cfl_speed(const Grid& G, const double* X, double* out, const RedWS& ws, hipStream_t s) {
  int b = red_blocks(G.N);
  if (G.nd == 2) k_cfl_speed<2><<<b, kBlock, 0, s>>>(G, X, out, ws);
  else k_cfl_speed<3><<<b, kBlock, 0, s>>>(G, X, out, ws);
  finalize<OpMax>(ws, b, 1, out, s);
}

// the maximum of the partials (the same combination as k_finalize) turned into the time step
// num / max on the device, num = cfl * min_d dx_d
__global__ void __launch_bounds__(kBlock) k_finalize_cfl_dt(const double* part, int nb, double num, double* dt) {
  __shared__ double sm[kBlock / 64];
  const double m = finalize_one<OpMax>(part, nb, 1, 0, sm);
  if (threadIdx.x == 0) *dt = num / m;
}

int cfl_partials(const Grid& G) { return red_blocks(G.N); }

void launch_cfl_dt_dev(const Grid& G, const double* X, double num, double* part, double* dt, hipStream_t s) {
  const int b = red_blocks(G.N);
  RedWS ws;
  ws.part = part;
  if (G.nd == 2) k_cfl_speed<2><<<b, kBlock, 0, s>>>(G, X, nullptr, ws);
  else k_cfl_speed<3><<<b, kBlock, 0, s>>>(G, X, nullptr, ws);
  k_finalize_cfl_dt<<<1, kBlock, 0, s>>>(part, b, num, dt);
}

}  // namespace jfnk
