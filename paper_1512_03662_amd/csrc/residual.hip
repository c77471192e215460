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
// Ideal gas with R = mu = 1: p = (gamma-1) rho e, T = (gamma-1) e.
//
// One thread per cell produces all nvar rows of that cell.  The scalar type is double for
// values, dual for the exact forward-mode product (branches frozen at the value), and the
// finite-difference product evaluates F at X + delta V with delta of eq. pert_old.
#include "common.hpp"
#include "kernels.hpp"
#include "probe.hpp"

namespace jfnk {

template <class T>
struct LoadVal {  // T(X)
  const double* X;
  int N;
  __device__ __forceinline__ T operator()(int var, int idx, double s) const {
    return T(s * X[var * N + idx]);
  }
};
struct LoadDual {  // dual(X, V)
  const double* X;
  const double* V;
  int N;
  __device__ __forceinline__ dual operator()(int var, int idx, double s) const {
    return dual(s * X[var * N + idx], s * V[var * N + idx]);
  }
};
struct LoadShift {  // X + delta V
  const double* X;
  const double* V;
  double delta;
  int N;
  __device__ __forceinline__ double operator()(int var, int idx, double s) const {
    return s * (X[var * N + idx] + delta * V[var * N + idx]);
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
  __device__ __forceinline__ T chi(T T_) const {
    if (G.chi_model == 1) return T(G.chi0);
    return G.chi0 * powr(T_ * G.chi_tref_inv, G.chi_exp);
  }
  // mass flux f_d and optionally energy flux g_d at the low-d face of c+o
  __device__ __forceinline__ T mass(int d, Off o) const {
    T w = u(d, o);
    T rs = upwind(rho(shift(o, d, -2)), rho(shift(o, d, -1)), rho(o), rho(shift(o, d, 1)), val(w));
    return w * rs;
  }
  __device__ __forceinline__ void mass_energy(int d, Off o, T* f, T* g) const {
    T w = u(d, o);
    double wv = val(w);
    T rs = upwind(rho(shift(o, d, -2)), rho(shift(o, d, -1)), rho(o), rho(shift(o, d, 1)), wv);
    T es = upwind(e(shift(o, d, -2)), e(shift(o, d, -1)), e(o), e(shift(o, d, 1)), wv);
    *f = w * rs;
    *g = (*f) * es;
  }
  __device__ __forceinline__ T cond(int d, Off o) const {
    if (G.bc[d] == 1) {
      int fi = P.c[d] + o.o[d];
      if (fi == 0) return T(G.qwall[d][0]);
      if (fi == G.n[d]) return T(G.qwall[d][1]);
    }
    double gm1 = G.gamma - 1.0;
    T Tm = gm1 * e(shift(o, d, -1));
    T T0 = gm1 * e(o);
    T chif = 0.5 * (chi(Tm) + chi(T0));
    return chif * (T0 - Tm) * G.idx[d];
  }
};

template <int ND, class T, class LD>
__device__ __forceinline__ void cell_R(const Grid& G, const Pos& P, const LD& ld, T* R) {
  Stencil<ND, T, LD> S(G, P, ld);
  const Off o = off0();
  const double gm1 = G.gamma - 1.0;
  T f0[ND], f1[ND], fm[ND];
  T rho0 = S.rho(o);
  T e0 = S.e(o);
  T p0 = gm1 * rho0 * e0;
  T Rrho = T(0.0), RE = T(0.0), divu = T(0.0);
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    T g0, g1;
    S.mass_energy(d, o, &f0[d], &g0);
    S.mass_energy(d, shift(o, d, 1), &f1[d], &g1);
    Rrho = Rrho - (f1[d] - f0[d]) * G.idx[d];
    RE = RE - (g1 - g0) * G.idx[d];
    divu = divu + (S.u(d, shift(o, d, 1)) - S.u(d, o)) * G.idx[d];
  }
  RE = RE - p0 * divu;
  if (G.chi_model != 0) {
#pragma unroll
    for (int d = 0; d < ND; ++d) RE = RE + (S.cond(d, shift(o, d, 1)) - S.cond(d, o)) * G.idx[d];
  }
  R[0] = Rrho;
  R[1] = RE;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    if (G.bc[d] == 1 && P.c[d] == 0) {
      R[2 + d] = T(0.0);
      continue;
    }
    fm[d] = S.mass(d, shift(o, d, -1));
    // Phi_dd at the centres of c and c - e_d
    T m0 = 0.5 * (f0[d] + f1[d]);
    T mm = 0.5 * (fm[d] + f0[d]);
    T um2 = S.u(d, shift(o, d, -2)), um1 = S.u(d, shift(o, d, -1)), u00 = S.u(d, o);
    T up1 = S.u(d, shift(o, d, 1)), up2 = S.u(d, shift(o, d, 2));
    T Pc0 = m0 * upwind(um1, u00, up1, up2, val(m0));
    T Pcm = mm * upwind(um2, um1, u00, up1, val(mm));
    T acc = -(Pc0 - Pcm) * G.idx[d];
#pragma unroll
    for (int e = 0; e < ND; ++e) {
      if (e == d) continue;
      // Phi_de at the (low-d, low-e) edges of c and c + e_e
      Off oe = shift(o, e, 1);
      T fa = S.mass(e, shift(o, d, -1));      // f_e[c - e_d]
      T fb = S.mass(e, shift(oe, d, -1));     // f_e[c - e_d + e_e]
      T me0 = 0.5 * (fa + f0[e]);
      T me1 = 0.5 * (fb + f1[e]);
      T vm2 = S.u(d, shift(o, e, -2)), vm1 = S.u(d, shift(o, e, -1));
      T vp1 = S.u(d, shift(o, e, 1)), vp2 = S.u(d, shift(o, e, 2));
      T Pe0 = me0 * upwind(vm2, vm1, u00, vp1, val(me0));
      T Pe1 = me1 * upwind(vm1, u00, vp1, vp2, val(me1));
      acc = acc - (Pe1 - Pe0) * G.idx[e];
    }
    T rhom = S.rho(shift(o, d, -1));
    T pm = gm1 * rhom * S.e(shift(o, d, -1));
    acc = acc - (p0 - pm) * G.idx[d] + 0.5 * (rhom + rho0) * G.g[d];
    R[2 + d] = acc;
  }
}

// U(X) at the cell with the stored (not ghosted) face velocity.
template <int ND, class T, class LD>
__device__ __forceinline__ void cell_U(const Grid& G, const Pos& P, const LD& ld, T* U) {
  Stencil<ND, T, LD> S(G, P, ld);
  const Off o = off0();
  T rho0 = S.rho(o);
  U[0] = rho0;
  U[1] = rho0 * S.e(o);
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    T rf = 0.5 * (S.rho(shift(o, d, -1)) + rho0);
    U[2 + d] = rf * ld(2 + d, P.lin, 1.0);
  }
}

// L (residual scaling) of the rows of one cell, from X (Sect. 4.1).
template <int ND>
__device__ __forceinline__ void cell_L(const Grid& G, const Pos& P, const double* X, double alpha1,
                                       double* L) {
  LoadVal<double> ld{X, G.N};
  Stencil<ND, double, LoadVal<double>> S(G, P, ld);
  const Off o = off0();
  double rho0 = S.rho(o), e0 = S.e(o);
  double k = G.gamma * (G.gamma - 1.0);
  double cs0 = sqrt(k * e0);
  L[0] = rho0;
  L[1] = rho0 * e0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    Off m = shift(o, d, -1);
    double csf = 0.5 * (sqrt(k * S.e(m)) + cs0);
    double rf = 0.5 * (S.rho(m) + rho0);
    double au = fabs(X[(2 + d) * G.N + P.lin]);
    L[2 + d] = rf * fmax(au, alpha1 * csf);
  }
}

// R (unknown scaling) of the unknowns of one cell, from X (Sect. 4.1).
template <int ND>
__device__ __forceinline__ void cell_Rs(const Grid& G, const Pos& P, const double* X, double alpha2,
                                        double* Rs) {
  LoadVal<double> ld{X, G.N};
  Stencil<ND, double, LoadVal<double>> S(G, P, ld);
  const Off o = off0();
  double e0 = S.e(o);
  double k = G.gamma * (G.gamma - 1.0);
  double cs0 = sqrt(k * e0);
  Rs[0] = S.rho(o);
  Rs[1] = e0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    double csf = 0.5 * (sqrt(k * S.e(shift(o, d, -1))) + cs0);
    double au = fabs(X[(2 + d) * G.N + P.lin]);
    Rs[2 + d] = fmax(au, alpha2 * csf);
  }
}

// ---- kernels --------------------------------------------------------------------------
template <int ND>
__global__ void __launch_bounds__(kBlock) k_resid_value(Grid G, ResidArgs a) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (lin >= G.N) return;
  Pos P = make_pos<ND>(G, lin);
  LoadVal<double> ld{a.X, G.N};
  double R[2 + ND], U[2 + ND], L[2 + ND];
  cell_R<ND>(G, P, ld, R);
  cell_U<ND>(G, P, ld, U);
  if (a.scaleL) cell_L<ND>(G, P, a.X, a.alpha1, L);
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

template <int ND>
__global__ void __launch_bounds__(kBlock) k_resid_tangent(Grid G, ResidArgs a) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (lin >= G.N) return;
  Pos P = make_pos<ND>(G, lin);
  LoadDual ld{a.X, a.V, G.N};
  dual R[2 + ND], U[2 + ND];
  double L[2 + ND];
  cell_R<ND>(G, P, ld, R);
  cell_U<ND>(G, P, ld, U);
  if (a.scaleL) cell_L<ND>(G, P, a.X, a.alpha1, L);
#pragma unroll
  for (int v = 0; v < 2 + ND; ++v) {
    double out = a.cU * U[v].d + a.cR * R[v].d;
    if (a.scaleL) out /= L[v];
    a.out[v * G.N + lin] = out;
  }
}

template <int ND>
__global__ void __launch_bounds__(kBlock) k_resid_fd(Grid G, ResidArgs a) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (lin >= G.N) return;
  const double xn2 = a.fd_norms[0], zn2 = a.fd_norms[1];
  double L[2 + ND];
  if (a.scaleL) {
    Pos P0 = make_pos<ND>(G, lin);
    cell_L<ND>(G, P0, a.X, a.alpha1, L);
  }
  if (!(zn2 > 0.0)) {
#pragma unroll
    for (int v = 0; v < 2 + ND; ++v) a.out[v * G.N + lin] = 0.0;
    return;
  }
  const double lam = a.fd_lambda;
  const double delta = lam * (lam + sqrt(xn2) / sqrt(zn2));
  Pos P = make_pos<ND>(G, lin);
  LoadShift ld{a.X, a.V, delta, G.N};
  double R[2 + ND], U[2 + ND];
  cell_R<ND>(G, P, ld, R);
  cell_U<ND>(G, P, ld, U);
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
  if (which == 0) cell_L<ND>(G, P, X, alpha, S);
  else cell_Rs<ND>(G, P, X, alpha, S);
#pragma unroll
  for (int v = 0; v < 2 + ND; ++v) {
    double x = in[v * G.N + lin];
    out[v * G.N + lin] = mode == 0 ? x / S[v] : x * S[v];
  }
}

// ---- launchers ------------------------------------------------------------------------
static inline dim3 cells_grid(const Grid& G) { return dim3((G.N + kBlock - 1) / kBlock); }

void launch_resid(const Grid& G, const ResidArgs& a, int mode, hipStream_t s) {
  dim3 gr = cells_grid(G), bl(kBlock);
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
  }
  if (G.nd == 2) {
    if (mode == 0) launch_k(fam, bytes, k_resid_value<2>, gr, bl, 0, s, G, a);
    else if (mode == 1) launch_k(fam, bytes, k_resid_tangent<2>, gr, bl, 0, s, G, a);
    else launch_k(fam, bytes, k_resid_fd<2>, gr, bl, 0, s, G, a);
  } else {
    if (mode == 0) launch_k(fam, bytes, k_resid_value<3>, gr, bl, 0, s, G, a);
    else if (mode == 1) launch_k(fam, bytes, k_resid_tangent<3>, gr, bl, 0, s, G, a);
    else launch_k(fam, bytes, k_resid_fd<3>, gr, bl, 0, s, G, a);
  }
}

void launch_scale_LR(const Grid& G, const double* X, double alpha, int which, const double* in,
                     double* out, int mode, hipStream_t s) {
  dim3 gr = cells_grid(G), bl(kBlock);
  if (G.nd == 2) k_scale_LR<2><<<gr, bl, 0, s>>>(G, X, alpha, which, in, out, mode);
  else k_scale_LR<3><<<gr, bl, 0, s>>>(G, X, alpha, which, in, out, mode);
}

}  // namespace jfnk
