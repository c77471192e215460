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
  double a_rad;     // radiation constant of the equation of state (0: ideal gas)
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

// ------------------------------------------------------------------------------------
// Equation of state (Sect. 2, App. A), R = mu = 1.
//   a_rad = 0: ideal gas, p = (gamma-1) rho e, T = (gamma-1) e, Gamma1 = Gamma3 = gamma.
//   a_rad > 0: gas + radiation in the diffusion limit, p = rho T + a T^4/3 and
//              e = c_v T + a T^4/rho with c_v = 1/(gamma-1) and a = a_rad.
// T(rho, e) is the positive root of c_v T + (a/rho) T^4 = e.  Newton steps start from
// min((gamma-1) e, (rho e/a)^(1/4)), which lies above the root by at most 38%; the quartic
// is convex, so the steps decrease to the root with relative error eps' <= 1.5 eps^2 and
// kEosNewton steps leave it at rounding (six would do).
// Kernels on the hot path take the choice as a template argument RAD, so that their ideal-gas
// instantiation carries no radiative code; the others branch on a_rad (uniform per launch).
// ------------------------------------------------------------------------------------
constexpr int kEosNewton = 8;

__device__ __forceinline__ double rad_temperature(const Grid& G, double rho, double e) {
  const double cv = 1.0 / (G.gamma - 1.0);
  const double b = G.a_rad / rho;
  double t = fmin((G.gamma - 1.0) * e, sqrt(sqrt(e / b)));
#pragma unroll
  for (int k = 0; k < kEosNewton; ++k) {
    const double t3 = t * t * t;
    t -= (cv * t + b * t3 * t - e) / (cv + 4.0 * b * t3);
  }
  return t;
}

template <bool RAD>
__device__ __forceinline__ double eos_T(const Grid& G, double rho, double e) {
  if constexpr (RAD) return rad_temperature(G, rho, e);
  else return (G.gamma - 1.0) * e;
}
// tangent: dT = (de + (a T^4/rho^2) drho) / (c_v + 4 a T^3/rho)
template <bool RAD>
__device__ __forceinline__ dual eos_T(const Grid& G, dual rho, dual e) {
  if constexpr (RAD) {
    const double t = rad_temperature(G, rho.v, e.v);
    const double b = G.a_rad / rho.v, t3 = t * t * t;
    return dual(t, (e.d + b * t3 * t / rho.v * rho.d) / (1.0 / (G.gamma - 1.0) + 4.0 * b * t3));
  } else {
    return (G.gamma - 1.0) * e;
  }
}

template <bool RAD, class T>
__device__ __forceinline__ T eos_p(const Grid& G, T rho, T e) {
  if constexpr (RAD) {
    const T t = eos_T<true>(G, rho, e);
    const T t2 = t * t;
    return rho * t + (G.a_rad / 3.0) * (t2 * t2);
  } else {
    return (G.gamma - 1.0) * rho * e;
  }
}

// p, T and the derivatives the preconditioner's transforms and the adjoint need:
// dp/drho|_e, dp/de|_rho, Gamma1 = (rho/p)(dp/drho|_e + (p/rho^2) dp/de|_rho),
// c_v = de/dT|_rho, dT/drho|_e, dT/de|_rho
struct Thermo {
  double p, T, dpdr, dpde, G1, cv, dTdr, dTde;
};

template <bool RAD>
__device__ __forceinline__ Thermo thermo(const Grid& G, double rho, double e) {
  Thermo s;
  const double gm1 = G.gamma - 1.0;
  if constexpr (!RAD) {
    s.p = gm1 * rho * e;
    s.T = gm1 * e;
    s.dpdr = gm1 * e;
    s.dpde = gm1 * rho;
    s.G1 = G.gamma;
    s.cv = 1.0 / gm1;
    s.dTdr = 0.0;
    s.dTde = gm1;
  } else {
    const double a = G.a_rad;
    const double t = rad_temperature(G, rho, e);
    const double t3 = t * t * t;
    const double eT = 1.0 / gm1 + 4.0 * a * t3 / rho;  // de/dT|_rho
    const double pT = rho + (4.0 / 3.0) * a * t3;      // dp/dT|_rho
    s.T = t;
    s.p = rho * t + (a / 3.0) * t3 * t;
    s.cv = eT;
    s.dTde = 1.0 / eT;
    s.dTdr = a * t3 * t / (rho * rho) * s.dTde;       // -(de/drho|_T) / (de/dT|_rho)
    s.dpde = pT * s.dTde;
    s.dpdr = t + pT * s.dTdr;
    s.G1 = (rho / s.p) * (s.dpdr + s.p / (rho * rho) * s.dpde);
  }
  return s;
}
__device__ __forceinline__ Thermo thermo_rt(const Grid& G, double rho, double e) {
  return G.a_rad == 0.0 ? thermo<false>(G, rho, e) : thermo<true>(G, rho, e);
}

// adiabatic sound speed sqrt(Gamma1 p/rho)
template <bool RAD>
__device__ __forceinline__ double sound_speed(const Grid& G, double rho, double e) {
  if constexpr (!RAD) {
    return sqrt(G.gamma * (G.gamma - 1.0) * e);
  } else {
    const Thermo s = thermo<true>(G, rho, e);
    return sqrt(s.dpdr + s.p / (rho * rho) * s.dpde);
  }
}
__device__ __forceinline__ double sound_speed_rt(const Grid& G, double rho, double e) {
  return G.a_rad == 0.0 ? sound_speed<false>(G, rho, e) : sound_speed<true>(G, rho, e);
}

// a * b rounded once and never fused into a neighbouring add (bit for bit the product a
// kernel would have stored); used where a vector is read scaled instead of being stored so
__device__ __forceinline__ double mul_nc(double a, double b) {
#pragma clang fp contract(off)
  return a * b;
}
// element i of a basis vector that is kept unnormalised: v[i] / ||v|| read as the product with
// sc = 1 / sqrt(||v||^2) (as the normalising kernel forms it), or v[i] when sc = 0
__device__ __forceinline__ double vread(const double* v, int i, double sc) {
  return sc != 0.0 ? mul_nc(v[i], sc) : v[i];
}
__device__ __forceinline__ double inv_norm(const double* nrm2) { return nrm2 ? 1.0 / sqrt(*nrm2) : 0.0; }

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
