// Device-side building blocks shared by the kernels of the implicit-step library (gfx950).
//
// Layout: structure-of-arrays FP64 fields, field v of cell (i,j,k) at v*N + i + nx*(j + ny*k).
// rho, e at cell centres; u_d on the low-d face of the cell (Sect. 2, staggered grid).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jfnk {

constexpr int kMaxDim = 3;
constexpr int kBlock = 256;

struct Grid {
  int nd;
  int n[3];
  int N;            // cells
  int stride[3];    // 1, nx, nx*ny
  int bc[3];        // 0 periodic, 1 wall
  double dx[3];
  double idx[3];    // 1/dx
  double gamma;
  double g[3];
  int chi_model;    // 0 none, 1 const, 2 power
  double chi0, chi_tref_inv, chi_exp;
  double qwall[3][2];
  double theta;
};

// ------------------------------------------------------------------------------------
// Forward-mode dual number: value and one tangent.
// ------------------------------------------------------------------------------------
struct dual {
  double v, d;
  __device__ __forceinline__ dual() = default;
  __device__ __forceinline__ constexpr dual(double a) : v(a), d(0.0) {}
  __device__ __forceinline__ constexpr dual(double a, double b) : v(a), d(b) {}
};
__device__ __forceinline__ dual operator+(dual a, dual b) { return dual(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ dual operator-(dual a, dual b) { return dual(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ dual operator-(dual a) { return dual(-a.v, -a.d); }
__device__ __forceinline__ dual operator*(dual a, dual b) {
  return dual(a.v * b.v, a.d * b.v + a.v * b.d);
}
__device__ __forceinline__ dual operator*(double s, dual a) { return dual(s * a.v, s * a.d); }
__device__ __forceinline__ dual operator*(dual a, double s) { return dual(s * a.v, s * a.d); }
__device__ __forceinline__ dual operator/(dual a, dual b) {
  double q = a.v / b.v;
  return dual(q, (a.d - q * b.d) / b.v);
}
__device__ __forceinline__ dual operator+(dual a, double s) { return dual(a.v + s, a.d); }

__device__ __forceinline__ double val(double a) { return a; }
__device__ __forceinline__ double val(dual a) { return a.v; }
__device__ __forceinline__ double tan_of(double) { return 0.0; }
__device__ __forceinline__ double tan_of(dual a) { return a.d; }

// x^p for positive x; p == 3 exactly takes the product form.
__device__ __forceinline__ double powr(double x, double p) {
  return p == 3.0 ? x * x * x : pow(x, p);
}
__device__ __forceinline__ dual powr(dual x, double p) {
  if (p == 3.0) {
    double x2 = x.v * x.v;
    return dual(x2 * x.v, 3.0 * x2 * x.d);
  }
  double y = pow(x.v, p);
  return dual(y, p * y / x.v * x.d);
}

// Reciprocal by the hardware estimate refined with two Newton steps (relative error within
// a few ulp; operands here are far from the overflow and denormal ranges).
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// van Leer (1974) harmonic slope: 2ab/(a+b) if ab > 0, else 0 (branch frozen for tangents).
// Evaluated without branches: the quotient is always formed and discarded by the select.
__device__ __forceinline__ double vl(double a, double b) {
  const double s = a + b;
  const double q = 2.0 * a * b * rcp_nr(s);
  return (a * b > 0.0) ? q : 0.0;
}
__device__ __forceinline__ dual vl(dual a, dual b) {
  const double s = a.v + b.v;
  const double r = rcp_nr(s);
  const double num = 2.0 * a.v * b.v;
  const double q = num * r;
  // d(2ab/(a+b)) = (2(a' b + a b') - q (a' + b')) / (a + b)
  const double dq = (2.0 * (a.d * b.v + a.v * b.d) - q * (a.d + b.d)) * r;
  const bool on = a.v * b.v > 0.0;
  return dual(on ? q : 0.0, on ? dq : 0.0);
}

// Upwind van Leer value at the face between q[c-1] (qm1) and q[c] (q0): w >= 0 takes the
// left-biased reconstruction qm1 + vl(qm1-qm2, q0-qm1)/2, else q0 - vl(q0-qm1, qp1-q0)/2.
// The operands are selected first so that one slope is evaluated without divergence.
template <class T>
__device__ __forceinline__ T sel(bool c, T a, T b) {
  return c ? a : b;
}
__device__ __forceinline__ dual sel(bool c, dual a, dual b) {
  return dual(c ? a.v : b.v, c ? a.d : b.d);
}
template <class T>
__device__ __forceinline__ T upwind(T qm2, T qm1, T q0, T qp1, double w) {
  const bool left = (w >= 0.0);
  const T d0 = q0 - qm1;
  const T base = sel(left, qm1, q0);
  const T a = sel(left, qm1 - qm2, d0);
  const T b = sel(left, d0, qp1 - q0);
  const double h = left ? 0.5 : -0.5;
  return base + h * vl(a, b);
}

// ------------------------------------------------------------------------------------
// Ghost rules per axis.  Periodic: wrap.  Wall: cell-centred and tangential quantities
// mirror evenly; the wall-normal velocity is zero on both wall faces, odd outside.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ int wrap(int i, int n) {
  if (i < 0) return i + n;
  if (i >= n) return i - n;
  return i;
}
__device__ __forceinline__ int ghost_even(int i, int n, int bc) {
  if (bc == 0) return wrap(i, n);
  if (i < 0) return -1 - i;
  if (i >= n) return 2 * n - 1 - i;
  return i;
}
// returns source index; *s = +1, -1 or 0
__device__ __forceinline__ int ghost_normal(int i, int n, int bc, double* s) {
  if (bc == 0) {
    *s = 1.0;
    return wrap(i, n);
  }
  if (i < 0) { *s = -1.0; return -i; }
  if (i > n) { *s = -1.0; return 2 * n - i; }
  if (i == 0 || i == n) { *s = 0.0; return 0; }
  *s = 1.0;
  return i;
}

// MI355X deals consecutive workgroups round-robin to its 8 XCDs, each with its own L2.
// Renumber them so that XCD k works on one contiguous range of blocks: neighbouring grid
// rows (the stencil's y and z neighbours) then share an L2.
constexpr int kNumXcd = 8;
__device__ __forceinline__ int xcd_block(int i, int nb) {
  const int q = nb / kNumXcd, r = nb % kNumXcd;
  const int x = i % kNumXcd, j = i / kNumXcd;
  return (x < r) ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
}

// Position of one thread's cell; loads of field var at an offset apply the ghost rules
// unless the whole radius-3 stencil is inside the grid ("interior").
struct Pos {
  int c[3];
  int lin;
  bool interior;
};

template <int ND>
__device__ __forceinline__ Pos make_pos(const Grid& G, int lin) {
  Pos p;
  p.lin = lin;
  int r = lin;
  p.c[0] = r % G.n[0];
  r /= G.n[0];
  p.c[1] = r % G.n[1];
  p.c[2] = r / G.n[1];
  bool in = true;
#pragma unroll
  for (int d = 0; d < ND; ++d) in = in && (p.c[d] >= 3) && (p.c[d] <= G.n[d] - 3);
  p.interior = in;
  return p;
}

// Offsets are packed as (ox, oy, oz).
struct Off {
  int o[3];
};
__device__ __forceinline__ Off off0() { return Off{{0, 0, 0}}; }
__device__ __forceinline__ Off shift(Off a, int d, int k) {
  a.o[d] += k;
  return a;
}

// index and sign of field var at offset; var >= 2 is velocity component var-2.  The axis
// loop is unrolled over the compile-time dimension so that positions stay in registers.
template <int ND>
__device__ __forceinline__ int gidx(const Grid& G, const Pos& p, int var, Off o, double* s) {
  if (p.interior) {
    *s = 1.0;
    int idx = p.lin + o.o[0] + o.o[1] * G.stride[1];
    if (ND == 3) idx += o.o[2] * G.stride[2];
    return idx;
  }
  double sign = 1.0;
  int idx = 0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    int i = p.c[d] + o.o[d];
    int src;
    if (var == 2 + d) {
      double sd;
      src = ghost_normal(i, G.n[d], G.bc[d], &sd);
      sign *= sd;
    } else {
      src = ghost_even(i, G.n[d], G.bc[d]);
    }
    idx += src * G.stride[d];
  }
  *s = sign;
  return idx;
}

}  // namespace jfnk
