// Residual F(X) = cU U(X) + cR R(X) - B of the time-discrete system and its directional
// derivatives (Sect. 2, eqs. cons1-cons3, mol, crank_nicholson; Sect. 4.2 eq. jacobian_free).
//
// Spatial operator R (staggered finite volumes with van Leer upwind fluxes, Sect. 2):
//   mass flux f_d = u_d rho*, energy flux g_d = f_d e* (rho*, e* upwind van Leer values at
//   the low-d face, left-biased when u_d >= 0), conductive flux q_d = chi_f (T[c]-T[c-1])/dx_d
//   (prescribed on wall faces);  R_rho = -div f,  R_E = -div g - p div u + div q;
//   momentum on the face control volume of u_d: Phi_dd at the cell centre carried by the
//   mean of f_d on both faces, Phi_de at the (low-d, low-e) edge carried by the mean of f_e
//   of the two cells sharing it, both with upwind van Leer values of u_d;
//   R_m,d = -ddiv Phi - (p[c]-p[c-1])/dx_d + rho_f g_d  (zero on wall-normal wall faces).
// Equation of state: ideal gas, or gas + radiation (RAD), with R = mu = 1 (common.hpp).
//
// Every flux is evaluated once per tile (see tile_axis); each thread then produces all nvar
// rows of its cell.  The scalar type is double for values, dual for the exact forward-mode
// product (branches frozen at the value), and the finite-difference product evaluates F at
// X + delta V with delta of eq. pert_old.
#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "probe.hpp"

namespace jfnk {

template <class T>
struct LoadVal {  // T(X)
  static constexpr bool kStage = false;
  const double* X;
  int N;
  __device__ __forceinline__ T operator()(int var, int idx, double s) const {
    return T(s * X[var * N + idx]);
  }
  __device__ __forceinline__ T operator()(int var, int idx) const { return T(X[var * N + idx]); }
};
struct LoadDual {  // dual(X, V)
  static constexpr bool kStage = false;
  const double* X;
  const double* V;
  int N;
  __device__ __forceinline__ dual operator()(int var, int idx, double s) const {
    return dual(s * X[var * N + idx], s * V[var * N + idx]);
  }
  __device__ __forceinline__ dual operator()(int var, int idx) const {
    return dual(X[var * N + idx], V[var * N + idx]);
  }
};
struct LoadShift {  // X + delta V
  static constexpr bool kStage = true;
  const double* X;
  const double* V;
  double delta;
  int N;
  __device__ __forceinline__ double operator()(int var, int idx, double s) const {
    return s * (X[var * N + idx] + delta * V[var * N + idx]);
  }
  __device__ __forceinline__ double operator()(int var, int idx) const {
    return X[var * N + idx] + delta * V[var * N + idx];
  }
};

template <int ND, class T, class LD>
struct Stencil {
  const Grid& G;
  const Pos& P;
  const LD& ld;
  __device__ Stencil(const Grid& g, const Pos& p, const LD& l) : G(g), P(p), ld(l) {}

  __device__ __forceinline__ T at(int var, Off o) const {
    double s;
    int i = gidx<ND>(G, P, var, o, &s);
    return ld(var, i, s);
  }
  __device__ __forceinline__ T rho(Off o) const { return at(0, o); }
  __device__ __forceinline__ T e(Off o) const { return at(1, o); }
  __device__ __forceinline__ T u(int d, Off o) const { return at(2 + d, o); }
};

// L (residual scaling) of the rows of one cell, from X (Sect. 4.1).
template <int ND, bool RAD>
__device__ __forceinline__ void cell_L(const Grid& G, const Pos& P, const double* X, double alpha1,
                                       double* L) {
  LoadVal<double> ld{X, G.N};
  Stencil<ND, double, LoadVal<double>> S(G, P, ld);
  const Off o = off0();
  double rho0 = S.rho(o), e0 = S.e(o);
  double cs0 = sound_speed<RAD>(G, rho0, e0);
  L[0] = rho0;
  L[1] = rho0 * e0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    Off m = shift(o, d, -1);
    double csf = 0.5 * (sound_speed<RAD>(G, S.rho(m), S.e(m)) + cs0);
    double rf = 0.5 * (S.rho(m) + rho0);
    double au = fabs(X[(2 + d) * G.N + P.lin]);
    L[2 + d] = rf * fmax(au, alpha1 * csf);
  }
}

// R (unknown scaling) of the unknowns of one cell, from X (Sect. 4.1).
template <int ND, bool RAD>
__device__ __forceinline__ void cell_Rs(const Grid& G, const Pos& P, const double* X, double alpha2,
                                        double* Rs) {
  LoadVal<double> ld{X, G.N};
  Stencil<ND, double, LoadVal<double>> S(G, P, ld);
  const Off o = off0();
  double e0 = S.e(o);
  double cs0 = sound_speed<RAD>(G, S.rho(o), e0);
  Rs[0] = S.rho(o);
  Rs[1] = e0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const Off m = shift(o, d, -1);
    double csf = 0.5 * (sound_speed<RAD>(G, S.rho(m), S.e(m)) + cs0);
    double au = fabs(X[(2 + d) * G.N + P.lin]);
    Rs[2 + d] = fmax(au, alpha2 * csf);
  }
}

// ---- tiled evaluation of R -------------------------------------------------------------
// One workgroup owns a tile of cells (32 x 8 in 2D, 8 x 8 x 4 in 3D; one cell per thread).
// Axis by axis it computes, once per face of the tile and of a one-cell halo, the mass flux
// f_D and the energy flux minus the conductive flux g_D - q_D into LDS; then, once per cell
// centre and edge, the momentum fluxes Phi_DD and Phi_eD (e != D) carried along D; finally
// every thread adds the D-differences of these fluxes to the rows of its own cell.  The
// state is read from memory through the caches (staging it in LDS with its radius-3 halo
// costs more occupancy than it saves); tiles whose footprint stays inside the grid skip the
// ghost rules.
template <int ND>
struct RTile;
template <>
struct RTile<2> {
  static constexpr int X = 32, Y = 8, Z = 1;
};
template <>
struct RTile<3> {
  static constexpr int X = 8, Y = 8, Z = 4;
};

template <int ND>
__host__ __device__ constexpr int tile_n(int i) {
  return i == 0 ? RTile<ND>::X : (i == 1 ? RTile<ND>::Y : RTile<ND>::Z);
}
// flux grid of axis D: faces [-1, T_D] along D, [-1, T_e - 1] along the other active axes
template <int ND, int D>
__host__ __device__ constexpr int fext(int i) {
  return i >= ND ? 1 : (i == D ? tile_n<ND>(i) + 2 : tile_n<ND>(i) + 1);
}
template <int ND>
__host__ __device__ constexpr int flo(int i) {
  return i >= ND ? 0 : -1;
}
// cell grid of axis D: [0, T_D] along D, [0, T_e - 1] along the others
template <int ND, int D>
__host__ __device__ constexpr int sext(int i) {
  return i == D ? tile_n<ND>(i) + 1 : tile_n<ND>(i);
}
template <int ND, int D>
__host__ __device__ constexpr int fsize() {
  return fext<ND, D>(0) * fext<ND, D>(1) * fext<ND, D>(2);
}
template <int ND, int D>
__host__ __device__ constexpr int ssize() {
  return sext<ND, D>(0) * sext<ND, D>(1) * sext<ND, D>(2);
}
__host__ __device__ constexpr int cmax(int a, int b) { return a > b ? a : b; }
template <int ND>
__host__ __device__ constexpr int fmaxsz() {
  return ND == 2 ? cmax(fsize<2, 0>(), fsize<2, 1>()) : cmax(fsize<3, 0>(), cmax(fsize<3, 1>(), fsize<3, 2>()));
}
template <int ND>
__host__ __device__ constexpr int smaxsz() {
  return ND == 2 ? cmax(ssize<2, 0>(), ssize<2, 1>()) : cmax(ssize<3, 0>(), cmax(ssize<3, 1>(), ssize<3, 2>()));
}
static_assert(RTile<2>::X * RTile<2>::Y * RTile<2>::Z == kBlock, "2D tile must have one cell per thread");
static_assert(RTile<3>::X * RTile<3>::Y * RTile<3>::Z == kBlock, "3D tile must have one cell per thread");

// index and sign of field var at tile-local coordinates q.  IN: the tile's radius-3
// footprint lies inside the grid (no ghost rules, sign 1).
template <int ND>
struct TileIdx {
  int o[3];
  int base;
  bool interior;
  template <bool IN>
  __device__ __forceinline__ int at(const Grid& G, int var, const int* q, double* s) const {
    if constexpr (IN) {
      *s = 1.0;
      int i = base + q[0] + q[1] * G.stride[1];
      if (ND == 3) i += q[2] * G.stride[2];
      return i;
    } else {
      double sign = 1.0;
      int idx = 0;
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        // coordinates of tiles that overhang the grid are clamped (those cells are not written)
        int i = min(max(o[d] + q[d], -3), G.n[d] + 2);
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
  }
};

template <int ND>
__device__ __forceinline__ TileIdx<ND> tile_setup(const Grid& G) {
  using TT = RTile<ND>;
  const int nbx = (G.n[0] + TT::X - 1) / TT::X, nby = (G.n[1] + TT::Y - 1) / TT::Y;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  TileIdx<ND> t;
  t.o[0] = (b % nbx) * TT::X;
  t.o[1] = ((b / nbx) % nby) * TT::Y;
  t.o[2] = (ND == 3) ? (b / (nbx * nby)) * TT::Z : 0;
  bool in = true;
#pragma unroll
  for (int d = 0; d < ND; ++d) in = in && (t.o[d] >= 4) && (t.o[d] + tile_n<ND>(d) + 3 <= G.n[d]);
  t.interior = in;
  t.base = t.o[0] + t.o[1] * G.stride[1] + ((ND == 3) ? t.o[2] * G.stride[2] : 0);
  return t;
}

template <class T>
__device__ __forceinline__ T chi_of(const Grid& G, T Tc) {
  if (G.chi_model == 1) return T(G.chi0);
  return G.chi0 * powr(Tc * G.chi_tref_inv, G.chi_exp);
}

// contributions of the fluxes along axis D to the rows R of the thread's own cell l
template <int ND, int D, bool RAD, class T, class AT>
__device__ __forceinline__ void tile_axis(const Grid& G, const AT& at, const TileIdx<ND>& ti, const int* l,
                                          bool own, T* R, T& divu, T* sF, T* sE, T* sP) {
  constexpr int E0 = fext<ND, D>(0), E1 = fext<ND, D>(1), E2 = fext<ND, D>(2);
  constexpr int NF = E0 * E1 * E2;
  constexpr int S0 = sext<ND, D>(0), S1 = sext<ND, D>(1), S2 = sext<ND, D>(2);
  constexpr int NS = S0 * S1 * S2;
  constexpr int SM = smaxsz<ND>();
  const int tid = threadIdx.x;
  const double ix = G.idx[D];
  auto fid = [&](const int* q) {
    return (q[0] - flo<ND>(0)) + (q[1] - flo<ND>(1)) * E0 + (q[2] - flo<ND>(2)) * E0 * E1;
  };
  auto sid = [&](const int* q) { return q[0] + q[1] * S0 + q[2] * S0 * S1; };
  // mass flux on the flux grid; energy minus conductive flux on the cell grid
  for (int p = tid; p < NF; p += kBlock) {
    int q[3] = {p % E0 + flo<ND>(0), (p / E0) % E1 + flo<ND>(1), p / (E0 * E1) + flo<ND>(2)};
    T r[4], ee[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int qq[3] = {q[0], q[1], q[2]};
      qq[D] += k - 2;
      r[k] = at(0, qq);
      ee[k] = at(1, qq);
    }
    const T w = at(2 + D, q);
    const double wv = val(w);
    const T f = w * upwind(r[0], r[1], r[2], r[3], wv);
    sF[p] = f;
    bool ins = q[D] >= 0;
#pragma unroll
    for (int e = 0; e < ND; ++e)
      if (e != D) ins = ins && q[e] >= 0;
    if (ins) {
      T gq = f * upwind(ee[0], ee[1], ee[2], ee[3], wv);
      if (G.chi_model != 0) {
        const int fi = ti.o[D] + q[D];
        T qc;
        if (G.bc[D] == 1 && fi == 0) {
          qc = T(G.qwall[D][0]);
        } else if (G.bc[D] == 1 && fi == G.n[D]) {
          qc = T(G.qwall[D][1]);
        } else {
          const T Tm = eos_T<RAD>(G, r[1], ee[1]), T0 = eos_T<RAD>(G, r[2], ee[2]);
          const T chif = 0.5 * (chi_of(G, Tm) + chi_of(G, T0));
          qc = chif * (T0 - Tm) * ix;
        }
        gq = gq - qc;
      }
      sE[sid(q)] = gq;
    }
  }
  __syncthreads();
  // momentum fluxes: Phi_DD at the centre of cell q - e_D, Phi_eD at the (low-e, low-D)
  // edge of cell q
  for (int p = tid; p < NS; p += kBlock) {
    int q[3] = {p % S0, (p / S0) % S1, p / (S0 * S1)};
    int k[3] = {q[0], q[1], q[2]};
    k[D] -= 1;
    const T m = 0.5 * (sF[fid(k)] + sF[fid(q)]);
    T u[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int kk[3] = {k[0], k[1], k[2]};
      kk[D] += j - 1;
      u[j] = at(2 + D, kk);
    }
    sP[p] = m * upwind(u[0], u[1], u[2], u[3], val(m));
    int slot = 1;
#pragma unroll
    for (int e = 0; e < ND; ++e) {
      if (e == D) continue;
      int qe[3] = {q[0], q[1], q[2]};
      qe[e] -= 1;
      const T me = 0.5 * (sF[fid(qe)] + sF[fid(q)]);
      T v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int qq[3] = {q[0], q[1], q[2]};
        qq[D] += j - 2;
        v[j] = at(2 + e, qq);
      }
      sP[slot * SM + p] = me * upwind(v[0], v[1], v[2], v[3], val(me));
      ++slot;
    }
  }
  __syncthreads();
  if (own) {
    int lp[3] = {l[0], l[1], l[2]};
    lp[D] += 1;
    R[0] = R[0] - (sF[fid(lp)] - sF[fid(l)]) * ix;
    R[1] = R[1] - (sE[sid(lp)] - sE[sid(l)]) * ix;
    divu = divu + (at(2 + D, lp) - at(2 + D, l)) * ix;
    R[2 + D] = R[2 + D] - (sP[sid(lp)] - sP[sid(l)]) * ix;
    int slot = 1;
#pragma unroll
    for (int e = 0; e < ND; ++e) {
      if (e == D) continue;
      R[2 + e] = R[2 + e] - (sP[slot * SM + sid(lp)] - sP[slot * SM + sid(l)]) * ix;
      ++slot;
    }
  }
  __syncthreads();
}

// box of the staged density and energy: tile-local coordinates [-3, T + 1] on every active
// axis (the reach of the face reconstructions and of the cell terms)
template <int ND>
__host__ __device__ constexpr int box_n(int i) {
  return i < ND ? tile_n<ND>(i) + 5 : 1;
}
template <int ND>
__host__ __device__ constexpr int box_size() {
  return box_n<ND>(0) * box_n<ND>(1) * box_n<ND>(2);
}

// sRE: LDS for rho and e on the box (value and finite-difference forms only; nullptr: read
// every field from memory)
template <int ND, bool IN, bool RAD, class T, class LD>
__device__ __forceinline__ bool tile_RU_in(const Grid& G, const LD& ld, const TileIdx<ND>& ti, T* R, T* U,
                                           int* lin_out, T* sF, T* sE, T* sP, T* sRE) {
  using TT = RTile<ND>;
  constexpr int BX = box_n<ND>(0), BY = box_n<ND>(1), BN = box_size<ND>();
  constexpr int BZ0 = (ND == 3) ? 3 : 0;
  const int t = threadIdx.x;
  auto atg = [&](int var, const int* q) -> T {
    double s;
    const int i = ti.template at<IN>(G, var, q, &s);
    if constexpr (IN) return ld(var, i);
    else return ld(var, i, s);
  };
  if (sRE) {
    for (int p = t; p < 2 * BN; p += kBlock) {
      const int var = p / BN, b = p - var * BN;
      const int q[3] = {b % BX - 3, (b / BX) % BY - 3, b / (BX * BY) - BZ0};
      sRE[p] = atg(var, q);
    }
    __syncthreads();
  }
  auto at = [&](int var, const int* q) -> T {
    if (var < 2 && sRE) return sRE[var * BN + (q[0] + 3) + (q[1] + 3) * BX + (q[2] + BZ0) * BX * BY];
    return atg(var, q);
  };
  const int l[3] = {t % TT::X, (t / TT::X) % TT::Y, t / (TT::X * TT::Y)};
  bool own = true;
#pragma unroll
  for (int d = 0; d < ND; ++d) own = own && (ti.o[d] + l[d] < G.n[d]);
#pragma unroll
  for (int v = 0; v < 2 + ND; ++v) R[v] = T(0.0);
  T divu = T(0.0);
  tile_axis<ND, 0, RAD>(G, at, ti, l, own, R, divu, sF, sE, sP);
  tile_axis<ND, 1, RAD>(G, at, ti, l, own, R, divu, sF, sE, sP);
  if constexpr (ND == 3) tile_axis<ND, 2, RAD>(G, at, ti, l, own, R, divu, sF, sE, sP);
  if (!own) return false;
  const T rho0 = at(0, l), e0 = at(1, l);
  const T p0 = eos_p<RAD>(G, rho0, e0);
  R[1] = R[1] - p0 * divu;
  const int lin = ti.base + l[0] + l[1] * G.stride[1] + ((ND == 3) ? l[2] * G.stride[2] : 0);
  U[0] = rho0;
  U[1] = rho0 * e0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    int lm[3] = {l[0], l[1], l[2]};
    lm[d] -= 1;
    const T rhom = at(0, lm);
    const T rf = 0.5 * (rhom + rho0);
    U[2 + d] = rf * ld(2 + d, lin, 1.0);  // the stored (not ghosted) face velocity
    if (G.bc[d] == 1 && ti.o[d] + l[d] == 0) {
      R[2 + d] = T(0.0);
    } else {
      const T pm = eos_p<RAD>(G, rhom, at(1, lm));
      R[2 + d] = R[2 + d] - (p0 - pm) * G.idx[d] + rf * G.g[d];
    }
  }
  *lin_out = lin;
  return true;
}

// R and U of the thread's cell; returns false (outputs unset) when the thread's cell lies
// outside the grid.  Every thread of the block must call it (it synchronises the block).
template <int ND, bool RAD, class T, class LD>
__device__ __forceinline__ bool tile_RU(const Grid& G, const LD& ld, T* R, T* U, int* lin_out) {
  // rho and e are staged in LDS when the loader combines two arrays per value (X + delta V);
  // for plain values the staging costs more than it saves, and staged duals would double
  // the LDS and halve the workgroups per CU
  constexpr bool STAGE = LD::kStage;
  __shared__ T sF[fmaxsz<ND>()];
  __shared__ T sE[smaxsz<ND>()];
  __shared__ T sP[ND * smaxsz<ND>()];
  __shared__ T sRE[STAGE ? 2 * box_size<ND>() : 1];
  T* re = STAGE ? sRE : nullptr;
  const TileIdx<ND> ti = tile_setup<ND>(G);
  if (ti.interior) return tile_RU_in<ND, true, RAD>(G, ld, ti, R, U, lin_out, sF, sE, sP, re);
  return tile_RU_in<ND, false, RAD>(G, ld, ti, R, U, lin_out, sF, sE, sP, re);
}

// ---- kernels --------------------------------------------------------------------------
template <int ND, bool RAD>
__global__ void __launch_bounds__(kBlock) k_resid_value(Grid G, ResidArgs a) {
  LoadVal<double> ld{a.X, G.N};
  double R[2 + ND], U[2 + ND], L[2 + ND];
  int lin;
  if (!tile_RU<ND, RAD>(G, ld, R, U, &lin)) return;
  if (a.scaleL) cell_L<ND, RAD>(G, make_pos<ND>(G, lin), a.X, a.alpha1, L);
#pragma unroll
  for (int v = 0; v < 2 + ND; ++v) {
    double gv = a.cU * U[v] + a.cR * R[v];
    if (a.G0) a.G0[v * G.N + lin] = gv;
    double b = a.B ? a.B[v * G.N + lin] : 0.0;
    double out = gv - b;
    if (a.scaleL) out /= L[v];
    a.out[v * G.N + lin] = out;
  }
}

template <int ND, bool RAD>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) k_resid_tangent(Grid G, ResidArgs a) {
  LoadDual ld{a.X, a.V, G.N};
  dual R[2 + ND], U[2 + ND];
  double L[2 + ND];
  int lin;
  if (!tile_RU<ND, RAD>(G, ld, R, U, &lin)) return;
  if (a.scaleL) cell_L<ND, RAD>(G, make_pos<ND>(G, lin), a.X, a.alpha1, L);
#pragma unroll
  for (int v = 0; v < 2 + ND; ++v) {
    double out = a.cU * U[v].d + a.cR * R[v].d;
    if (a.scaleL) out /= L[v];
    a.out[v * G.N + lin] = out;
  }
}

// Xs = X + delta V with delta of eq. pert_old from the device norms (0 when V = 0), the
// state at which the finite-difference product evaluates F
__global__ void __launch_bounds__(kBlock) k_fd_shift(size_t n, const double* X, const double* V,
                                                     const double* norms, double lam, double* Xs) {
  const double xn2 = norms[0], zn2 = norms[1];
  const double delta = (zn2 > 0.0) ? lam * (lam + sqrt(xn2) / sqrt(zn2)) : 0.0;
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
    Xs[i] = X[i] + delta * V[i];
}

// PRE: F is evaluated at the precomputed X + delta V in a.shift (one array per value, as
// for F itself); otherwise every load forms X + delta V from X and V
template <int ND, bool RAD, bool PRE>
__global__ void __launch_bounds__(kBlock) k_resid_fd(Grid G, ResidArgs a) {
  const double xn2 = a.fd_norms[0], zn2 = a.fd_norms[1];
  if (!(zn2 > 0.0)) {  // the same for every thread: no block-wide work follows
    const TileIdx<ND> ti = tile_setup<ND>(G);
    using TT = RTile<ND>;
    const int t = threadIdx.x;
    const int l[3] = {t % TT::X, (t / TT::X) % TT::Y, t / (TT::X * TT::Y)};
#pragma unroll
    for (int d = 0; d < ND; ++d)
      if (ti.o[d] + l[d] >= G.n[d]) return;
    const int lin = ti.base + l[0] + l[1] * G.stride[1] + ((ND == 3) ? l[2] * G.stride[2] : 0);
#pragma unroll
    for (int v = 0; v < 2 + ND; ++v) a.out[v * G.N + lin] = 0.0;
    return;
  }
  const double lam = a.fd_lambda;
  const double delta = lam * (lam + sqrt(xn2) / sqrt(zn2));
  using LD = std::conditional_t<PRE, LoadVal<double>, LoadShift>;
  LD ld = [&]() {
    if constexpr (PRE) return LoadVal<double>{a.shift, G.N};
    else return LoadShift{a.X, a.V, delta, G.N};
  }();
  double R[2 + ND], U[2 + ND], L[2 + ND];
  int lin;
  if (!tile_RU<ND, RAD>(G, ld, R, U, &lin)) return;
  if (a.scaleL) cell_L<ND, RAD>(G, make_pos<ND>(G, lin), a.X, a.alpha1, L);
#pragma unroll
  for (int v = 0; v < 2 + ND; ++v) {
    double out = (a.cU * U[v] + a.cR * R[v] - a.B[v * G.N + lin]) / delta;
    if (a.scaleL) out /= L[v];
    a.out[v * G.N + lin] = out;
  }
}

template <int ND>
__global__ void __launch_bounds__(kBlock) k_scale_LR(Grid G, const double* X, double alpha, int which,
                                                     const double* in, double* out, int mode) {
  // mode 0: out = in / S, mode 1: out = in * S, with S = L (which = 0) or R (which = 1)
  int lin = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (lin >= G.N) return;
  Pos P = make_pos<ND>(G, lin);
  double S[2 + ND];
  if (G.a_rad == 0.0) {
    if (which == 0) cell_L<ND, false>(G, P, X, alpha, S);
    else cell_Rs<ND, false>(G, P, X, alpha, S);
  } else {
    if (which == 0) cell_L<ND, true>(G, P, X, alpha, S);
    else cell_Rs<ND, true>(G, P, X, alpha, S);
  }
#pragma unroll
  for (int v = 0; v < 2 + ND; ++v) {
    double x = in[v * G.N + lin];
    out[v * G.N + lin] = mode == 0 ? x / S[v] : x * S[v];
  }
}

// ---- launchers ------------------------------------------------------------------------
static inline dim3 cells_grid(const Grid& G) { return dim3((G.N + kBlock - 1) / kBlock); }

template <int ND>
static dim3 tile_grid(const Grid& G) {
  int b = 1;
  for (int d = 0; d < ND; ++d) b *= (G.n[d] + tile_n<ND>(d) - 1) / tile_n<ND>(d);
  return dim3(b);
}

template <bool RAD>
static void launch_resid_k(const Grid& G, const ResidArgs& a, int mode, int fam, double bytes, dim3 gr,
                           dim3 bl, hipStream_t s) {
  const bool pre = a.shift != nullptr;
  if (G.nd == 2) {
    if (mode == 0) launch_k(fam, bytes, k_resid_value<2, RAD>, gr, bl, 0, s, G, a);
    else if (mode == 1) launch_k(fam, bytes, k_resid_tangent<2, RAD>, gr, bl, 0, s, G, a);
    else if (pre) launch_k(fam, bytes, k_resid_fd<2, RAD, true>, gr, bl, 0, s, G, a);
    else launch_k(fam, bytes, k_resid_fd<2, RAD, false>, gr, bl, 0, s, G, a);
  } else {
    if (mode == 0) launch_k(fam, bytes, k_resid_value<3, RAD>, gr, bl, 0, s, G, a);
    else if (mode == 1) launch_k(fam, bytes, k_resid_tangent<3, RAD>, gr, bl, 0, s, G, a);
    else if (pre) launch_k(fam, bytes, k_resid_fd<3, RAD, true>, gr, bl, 0, s, G, a);
    else launch_k(fam, bytes, k_resid_fd<3, RAD, false>, gr, bl, 0, s, G, a);
  }
}

void launch_resid(const Grid& G, const ResidArgs& a, int mode, hipStream_t s) {
  dim3 gr = (G.nd == 2) ? tile_grid<2>(G) : tile_grid<3>(G), bl(kBlock);
  // algorithmic bytes: every field read or written once (FP64)
  const double nvN = 8.0 * (2 + G.nd) * G.N;
  int fam;
  double bytes;
  if (mode == 0) {
    fam = KF_RESID_VALUE;
    bytes = nvN * (2 + (a.B ? 1 : 0) + (a.G0 ? 1 : 0));
  } else if (mode == 1) {
    fam = KF_RESID_TANGENT;
    bytes = nvN * 3;
  } else {
    fam = KF_RESID_FD;
    bytes = nvN * 4;
    if (a.shift) {
      const size_t n = (size_t)(2 + G.nd) * G.N;
      const int nb = (int)std::min<size_t>((n + kBlock - 1) / kBlock, 8192);
      launch_k(KF_FD_SHIFT, nvN * 3, k_fd_shift, dim3(nb), dim3(kBlock), 0, s, n, a.X, a.V, a.fd_norms,
               a.fd_lambda, a.shift);
    }
  }
  if (G.a_rad == 0.0) launch_resid_k<false>(G, a, mode, fam, bytes, gr, bl, s);
  else launch_resid_k<true>(G, a, mode, fam, bytes, gr, bl, s);
}

void launch_scale_LR(const Grid& G, const double* X, double alpha, int which, const double* in,
                     double* out, int mode, hipStream_t s) {
  dim3 gr = cells_grid(G), bl(kBlock);
  if (G.nd == 2) k_scale_LR<2><<<gr, bl, 0, s>>>(G, X, alpha, which, in, out, mode);
  else k_scale_LR<3><<<gr, bl, 0, s>>>(G, X, alpha, which, in, out, mode);
}

}  // namespace jfnk
