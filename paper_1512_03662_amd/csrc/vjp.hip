// Transposed Jacobian products of the residual, J^T w, in gather form (no atomics, so the
// result is deterministic), and the transposed physics-based preconditioner used by the
// adjoint of an implicit step.
//
// F = cU U(X) + cR R(X) - b with the staggered operator R of residual.hip.  The adjoint is
// taken with respect to a ghost-padded copy of X (3 ghost layers per side, ghost values
// treated as independent inputs), then folded back through the ghost rules (wrap, even
// mirror, odd mirror with zero on wall faces):
//   stage 0: the mass flux f_d on every padded face (stored, read by the next two stages);
//   stage A: adjoint of the mass flux f_d on every padded face, from w (R_rho, the energy
//            flux g = f e*, the momentum fluxes through their carrying mass flux);
//   stage B: adjoint of every padded input (rho, e, u_d): per tile, each reconstruction term
//            is differentiated once and its four partials reach their cells through LDS;
//   fold:    X_bar = cU (dU/dX)^T w + sum over the padded copies of each stored value.
// Terms whose adjoint weight is exactly zero are skipped, so only terms that the forward
// evaluates for some interior row are evaluated, with the same (in-range) ghost accesses.
#include "common.hpp"
#include "kernels.hpp"
#include "probe.hpp"

namespace jfnk {

struct PadGrid {
  int P[3];       // padded extents (n + 6 on used axes, 1 otherwise)
  int pstride[3];
  int PN;
};

static PadGrid make_pad(const Grid& G) {
  PadGrid p;
  for (int d = 0; d < 3; ++d) p.P[d] = (d < G.nd) ? G.n[d] + 6 : 1;
  p.pstride[0] = 1;
  p.pstride[1] = p.P[0];
  p.pstride[2] = p.P[0] * p.P[1];
  p.PN = p.P[0] * p.P[1] * p.P[2];
  return p;
}

// derivative of the upwind van Leer value w.r.t. its four arguments (qm2, qm1, q0, qp1),
// branch frozen at the value; evaluated without branches with one refined reciprocal (as
// the forward's vl).  Left (w >= 0): value qm1 + v/2 with a = qm1 - qm2, b = q0 - qm1;
// right: q0 - v/2 with a = q0 - qm1, b = qp1 - q0; v = 2ab/(a+b) when ab > 0, else 0, and
// dv/da = 2b^2/(a+b)^2, dv/db = 2a^2/(a+b)^2.
__device__ __forceinline__ double upwind_grad(double qm2, double qm1, double q0, double qp1, double w,
                                              double* g) {
  const bool left = (w >= 0.0);
  const double d0 = q0 - qm1;
  const double a = left ? (qm1 - qm2) : d0;
  const double b = left ? d0 : (qp1 - q0);
  const double r = rcp_nr(a + b);
  const bool on = a * b > 0.0;
  const double v = on ? 2.0 * a * b * r : 0.0;
  const double r2 = r * r;
  const double da = on ? 2.0 * b * b * r2 : 0.0;
  const double db = on ? 2.0 * a * a * r2 : 0.0;
  g[0] = left ? -0.5 * da : 0.0;
  g[1] = left ? 1.0 + 0.5 * (da - db) : 0.5 * da;
  g[2] = left ? 0.5 * db : 1.0 - 0.5 * (da - db);
  g[3] = left ? 0.0 : -0.5 * db;
  return left ? qm1 + 0.5 * v : q0 - 0.5 * v;
}

// Accesses at logical (possibly ghost) positions; same ghost rules as the forward.  IN:
// every position accessed lies inside the grid, away from wall faces (no ghost rules).
template <int ND, bool IN = false>
struct Acc {
  const Grid& G;
  const double* X;
  const double* w;   // adjoint seed (interior rows)
  double cR;
  __device__ Acc(const Grid& g, const double* x, const double* ww, double c) : G(g), X(x), w(ww), cR(c) {}

  __device__ __forceinline__ double x(int var, const int* c) const {
    if constexpr (IN) {
      int idx = c[0] + c[1] * G.stride[1];
      if (ND == 3) idx += c[2] * G.stride[2];
      return X[var * G.N + idx];
    }
    double sign = 1.0;
    int idx = 0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      int src;
      if (var == 2 + d) {
        double sd;
        src = ghost_normal(c[d], G.n[d], G.bc[d], &sd);
        sign *= sd;
      } else {
        src = ghost_even(c[d], G.n[d], G.bc[d]);
      }
      // the active terms only read logical positions in [-3, n+2], where the ghost rules
      // already land inside the grid; the clamp keeps every read in bounds regardless
      src = min(max(src, 0), G.n[d] - 1);
      idx += src * G.stride[d];
    }
    return sign * X[var * G.N + idx];
  }
  // seed of row (var, c) of the R part: zero outside the grid and on wall-normal wall faces
  __device__ __forceinline__ double W(int var, const int* c) const {
    if constexpr (IN) {
      int i = c[0] + c[1] * G.stride[1];
      if (ND == 3) i += c[2] * G.stride[2];
      return cR * w[var * G.N + i];
    }
    int idx = 0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      if (c[d] < 0 || c[d] >= G.n[d]) return 0.0;
      idx += c[d] * G.stride[d];
    }
    if (var >= 2) {
      int d = var - 2;
      if (G.bc[d] == 1 && c[d] == 0) return 0.0;
    }
    return cR * w[var * G.N + idx];
  }
  __device__ __forceinline__ double rho(const int* c) const { return x(0, c); }
  __device__ __forceinline__ double e(const int* c) const { return x(1, c); }
  __device__ __forceinline__ double u(int d, const int* c) const { return x(2 + d, c); }
};

#define SH(dst, src, d, k)           \
  int dst[3] = {src[0], src[1], src[2]}; \
  dst[d] += (k)

// mass flux f_d at the low-d face of logical cell c
template <int ND, class AC>
__device__ __forceinline__ double mflux(const AC& A, int d, const int* c) {
  SH(m2, c, d, -2);
  SH(m1, c, d, -1);
  SH(p1, c, d, 1);
  double w = A.u(d, c);
  return w * upwind(A.rho(m2), A.rho(m1), A.rho(c), A.rho(p1), w);
}

// padded index of logical cell q (coordinates clamped to the padded grid; every term that
// reads a stored mass flux lies inside it)
template <int ND>
__device__ __forceinline__ int pad_index(const PadGrid& PG, const int* q) {
  int idx = 0;
#pragma unroll
  for (int d = 0; d < ND; ++d) idx += min(max(q[d] + 3, 0), PG.P[d] - 1) * PG.pstride[d];
  return idx;
}

// ---- stage 0: mass flux f_d on every padded face (read by stages A and B) ----------------
template <int ND>
__global__ void __launch_bounds__(kBlock) k_vjp_flux(Grid G, PadGrid PG, const double* X, double* mf) {
  int pl = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (pl >= PG.PN) return;
  int c[3];
  c[0] = pl % PG.P[0] - 3;
  int r = pl / PG.P[0];
  c[1] = (ND >= 2) ? r % PG.P[1] - 3 : 0;
  c[2] = (ND == 3) ? r / PG.P[1] - 3 : 0;
  Acc<ND> A(G, X, nullptr, 0.0);
#pragma unroll
  for (int d = 0; d < ND; ++d) mf[(size_t)d * PG.PN + pl] = mflux<ND>(A, d, c);
}

// ---- stage B: adjoint of every padded input, tiled -----------------------------------------
// Every term of R that reads a field through a four-point upwind reconstruction along an axis
// A (the mass and energy fluxes along A, the momentum fluxes carried along A) is evaluated
// once per point of the tile's face grid along A: its four partial derivatives times the
// term's adjoint weight go to LDS, and each cell of the tile then adds the four entries that
// reach it (point q feeds the cells q - 2 .. q + 1 along A).  A tile of padded cells is
// 32 x 8 (2D) or 16 x 4 x 4 (3D); its face grid along A spans [-1, T_A + 2) (tile-local) along
// A and the tile along the other axes.  Terms local to a cell (pressure, gravity, the cell's
// own mass flux, div u) are added by the cell's thread.  Partial derivatives are taken with
// the upwind choices and limiter branches frozen, as in the forward.
template <int ND>
__host__ __device__ constexpr int bt(int d) {
  return ND == 2 ? (d == 0 ? 32 : (d == 1 ? 8 : 1)) : (d == 0 ? 16 : 4);
}
template <int ND, int A>
__host__ __device__ constexpr int bext(int i) {
  return i >= ND ? 1 : (i == A ? bt<ND>(i) + 3 : bt<ND>(i));
}
template <int ND, int A>
__host__ __device__ constexpr int bfaces() {
  return bext<ND, A>(0) * bext<ND, A>(1) * bext<ND, A>(2);
}
__host__ __device__ constexpr int bmax(int a, int b) { return a > b ? a : b; }
template <int ND>
__host__ __device__ constexpr int bfaces_max() {
  return ND == 2 ? bmax(bfaces<2, 0>(), bfaces<2, 1>())
                 : bmax(bfaces<3, 0>(), bmax(bfaces<3, 1>(), bfaces<3, 2>()));
}
static_assert(bt<2>(0) * bt<2>(1) == kBlock && bt<3>(0) * bt<3>(1) * bt<3>(2) == kBlock,
              "one padded cell per thread");

template <int ND>
static int btile_blocks(const PadGrid& PG) {
  int b = 1;
  for (int d = 0; d < 3; ++d) b *= (PG.P[d] + bt<ND>(d) - 1) / bt<ND>(d);
  return b;
}

// o: logical coordinates of the tile's first cell; interior: every access of the tile's
// terms (at most 5 cells beyond it) lies inside the grid, away from its walls
template <int ND>
struct BTile {
  int o[3];
  bool interior;
};
template <int ND>
__device__ __forceinline__ BTile<ND> btile_setup(const Grid& G, const PadGrid& PG) {
  int nb[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) nb[d] = (PG.P[d] + bt<ND>(d) - 1) / bt<ND>(d);
  const int b = xcd_block(blockIdx.x, gridDim.x);
  BTile<ND> t;
  t.o[0] = (b % nb[0]) * bt<ND>(0) - 3;
  t.o[1] = ((b / nb[0]) % nb[1]) * bt<ND>(1) - 3;
  t.o[2] = (ND == 3) ? (b / (nb[0] * nb[1])) * bt<ND>(2) - 3 : 0;
  bool in = true;
#pragma unroll
  for (int d = 0; d < ND; ++d) in = in && (t.o[d] >= 6) && (t.o[d] + bt<ND>(d) + 6 <= G.n[d]);
  t.interior = in;
  return t;
}

// one scatter pass along A with NS independent term sets: coef(f, g) fills g[s * 4 + j],
// the contribution of face point f (logical) to cell f + (j - 2) e_A of set s; acc[s] of the
// thread's own cell l receives the sum of what reaches it
template <int ND, int A, int NS, class CF>
__device__ __forceinline__ void bscatter(const BTile<ND>& T, const int* l, bool own, double* sC, const CF& coef,
                                         double* acc) {
  constexpr int E0 = bext<ND, A>(0), E1 = bext<ND, A>(1), E2 = bext<ND, A>(2);
  constexpr int NF = E0 * E1 * E2;
  constexpr int M = bfaces_max<ND>();
  for (int p = threadIdx.x; p < NF; p += kBlock) {
    int f[3] = {p % E0, (p / E0) % E1, p / (E0 * E1)};
    f[A] -= 1;
#pragma unroll
    for (int d = 0; d < 3; ++d) f[d] += T.o[d];
    double g[NS * 4];
    coef(f, g);
#pragma unroll
    for (int i = 0; i < NS * 4; ++i) sC[i * M + p] = g[i];
  }
  __syncthreads();
  if (own) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int q[3] = {l[0], l[1], l[2]};
      q[A] += 3 - j;  // face l + (2 - j) e_A, shifted by the face grid's origin -1
      const int p = q[0] + q[1] * E0 + q[2] * E0 * E1;
#pragma unroll
      for (int s = 0; s < NS; ++s) acc[s] += sC[(s * 4 + j) * M + p];
    }
  }
  __syncthreads();
}

// ---- stage A: adjoint of the mass flux f_d on every padded face, tiled ------------------
// fbar_d at face c takes R_rho's difference, the energy flux's e*, and half of each momentum
// flux term whose carrying mass flux averages f_d at c: Phi_dd at the centres c - e_d and c,
// Phi_ed (e != d) at the edges c and c + e_e.  Each of those terms is evaluated once per
// tile point into LDS; a face adds the two that reach it.
template <int ND, int B>
__host__ __device__ constexpr int pext(int i) {
  return i >= ND ? 1 : (i == B ? bt<ND>(i) + 1 : bt<ND>(i));
}
template <int ND, int B>
__host__ __device__ constexpr int ppoints() {
  return pext<ND, B>(0) * pext<ND, B>(1) * pext<ND, B>(2);
}
template <int ND>
__host__ __device__ constexpr int ppoints_max() {
  return ND == 2 ? bmax(ppoints<2, 0>(), ppoints<2, 1>())
                 : bmax(ppoints<3, 0>(), bmax(ppoints<3, 1>(), ppoints<3, 2>()));
}
// term values at points [LO, LO + T_B + 1) along B (tile-local; LO = -1 or 0); the thread's
// own cell l gets the sum of the entries at l and at l - e_B (LO = -1) or l + e_B (LO = 0)
template <int ND, int B, int LO, class VF>
__device__ __forceinline__ double bpair(const BTile<ND>& T, const int* l, bool own, double* sV, const VF& val) {
  constexpr int E0 = pext<ND, B>(0), E1 = pext<ND, B>(1), E2 = pext<ND, B>(2);
  constexpr int NP = E0 * E1 * E2;
  for (int p = threadIdx.x; p < NP; p += kBlock) {
    int f[3] = {p % E0, (p / E0) % E1, p / (E0 * E1)};
    f[B] += LO;
#pragma unroll
    for (int d = 0; d < 3; ++d) f[d] += T.o[d];
    sV[p] = val(f);
  }
  __syncthreads();
  double r = 0.0;
  if (own) {
    int q[3] = {l[0], l[1], l[2]};
    q[B] -= LO;
    const int i1 = q[0] + q[1] * E0 + q[2] * E0 * E1;
    q[B] += (LO == -1) ? -1 : 1;
    const int i2 = q[0] + q[1] * E0 + q[2] * E0 * E1;
    r = sV[i1] + sV[i2];
  }
  __syncthreads();
  return r;
}

template <int ND, int D, class AC>
__device__ __forceinline__ double vjp_faceA(const Grid& G, const PadGrid& PG, const AC& Ac, const BTile<ND>& T,
                                            const int* l, const int* c, bool own, const double* mf, double* sV) {
  const double ih = G.idx[D];
  auto MF = [&](int d, const int* q) { return mf[(size_t)d * PG.PN + pad_index<ND>(PG, q)]; };
  // Phi_DD at the centre between faces cc and cc + e_D, for cc = c - e_D and c
  double fb = bpair<ND, D, -1>(T, l, own, sV, [&](const int* cc) -> double {
    SH(cp, cc, D, 1);
    const double Pb = (Ac.W(2 + D, cp) - Ac.W(2 + D, cc)) * ih;
    if (Pb == 0.0) return 0.0;
    const double m = 0.5 * (MF(D, cc) + MF(D, cp));
    SH(um1, cc, D, -1);
    SH(up2, cc, D, 2);
    return 0.5 * Pb * upwind(Ac.u(D, um1), Ac.u(D, cc), Ac.u(D, cp), Ac.u(D, up2), m);
  });
  // Phi_eD (u_e carried along D) at the edges ce = c and c + e_e
#pragma unroll
  for (int e = 0; e < ND; ++e) {
    if (e == D) continue;
    auto val = [&](const int* ce) -> double {
      SH(ced, ce, D, -1);
      const double Pb = (Ac.W(2 + e, ce) - Ac.W(2 + e, ced)) * ih;
      if (Pb == 0.0) return 0.0;
      SH(cee, ce, e, -1);
      const double m = 0.5 * (MF(D, cee) + MF(D, ce));
      SH(d2, ce, D, -2);
      SH(dp, ce, D, 1);
      return 0.5 * Pb * upwind(Ac.u(e, d2), Ac.u(e, ced), Ac.u(e, ce), Ac.u(e, dp), m);
    };
    if (e == 0) fb += bpair<ND, 0, 0>(T, l, own, sV, val);
    else if (e == 1) fb += bpair<ND, 1, 0>(T, l, own, sV, val);
    else fb += bpair<ND, (ND == 3 ? 2 : 1), 0>(T, l, own, sV, val);
  }
  if (!own) return 0.0;
  // R_rho's difference and the energy flux g_D = f_D e*
  SH(cm, c, D, -1);
  fb += (Ac.W(0, c) - Ac.W(0, cm)) * ih;
  const double gb = (Ac.W(1, c) - Ac.W(1, cm)) * ih;
  if (gb != 0.0) {
    SH(m2, c, D, -2);
    SH(p1, c, D, 1);
    fb += gb * upwind(Ac.e(m2), Ac.e(cm), Ac.e(c), Ac.e(p1), Ac.u(D, c));
  }
  return fb;
}

template <int ND, class AC>
__device__ __forceinline__ void vjp_tileA(const Grid& G, const PadGrid& PG, const AC& Ac, const BTile<ND>& T,
                                          const double* mf, double* fbar, double* sV) {
  const int t = threadIdx.x;
  const int l[3] = {t % bt<ND>(0), (t / bt<ND>(0)) % bt<ND>(1), t / (bt<ND>(0) * bt<ND>(1))};
  int c[3], pl = 0;
  bool own = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    c[d] = T.o[d] + l[d];
    if (d < ND) {
      own = own && (c[d] + 3 < PG.P[d]);
      pl += (c[d] + 3) * PG.pstride[d];
    }
  }
  const double f0 = vjp_faceA<ND, 0>(G, PG, Ac, T, l, c, own, mf, sV);
  const double f1 = vjp_faceA<ND, 1>(G, PG, Ac, T, l, c, own, mf, sV);
  double f2 = 0.0;
  if constexpr (ND == 3) f2 = vjp_faceA<ND, 2>(G, PG, Ac, T, l, c, own, mf, sV);
  if (!own) return;
  fbar[pl] = f0;
  fbar[(size_t)PG.PN + pl] = f1;
  if constexpr (ND == 3) fbar[(size_t)2 * PG.PN + pl] = f2;
}

template <int ND>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) k_vjp_stageA(Grid G, PadGrid PG, const double* X, const double* w,
                                                       double cR, const double* mf, double* fbar) {
  __shared__ double sV[ppoints_max<ND>()];
  const BTile<ND> T = btile_setup<ND>(G, PG);
  if (T.interior) vjp_tileA<ND>(G, PG, Acc<ND, true>(G, X, w, cR), T, mf, fbar, sV);
  else vjp_tileA<ND>(G, PG, Acc<ND, false>(G, X, w, cR), T, mf, fbar, sV);
}

// the passes along axis A: mass and energy fluxes (to rho, e), Phi_AA (to u_A), and Phi_dA
// for d != A (u_d carried along A, to u_d)
template <int ND, int A, bool RAD, class AC>
__device__ __forceinline__ void vjp_axisB(const Grid& G, const PadGrid& PG, const AC& Ac, const BTile<ND>& T,
                                          const int* l, bool own, const double* mf, const double* fbar,
                                          double* sC, double& rb, double& eb, double* ub) {
  const double ih = G.idx[A];
  const double gm1 = G.gamma - 1.0;
  auto MF = [&](int d, const int* q) { return mf[(size_t)d * PG.PN + pad_index<ND>(PG, q)]; };
  auto padded = [&](const int* q) -> int {
    int idx = 0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const int pq = q[d] + 3;
      if (pq < 0 || pq >= PG.P[d]) return -1;
      idx += pq * PG.pstride[d];
    }
    return idx;
  };
  {
    // Each term's weight is tested only after all of the point's loads have been issued
    // (every index is in range on every path), and a term of weight zero is dropped by a
    // select: the loads of a point are then one batch instead of a chain of round trips
    // behind the weight tests.
    auto coef = [&](const int* f, double* g) {
      SH(m2, f, A, -2);
      SH(m1, f, A, -1);
      SH(p1, f, A, 1);
      const int pf = padded(f);
      const double wv = Ac.u(A, f);
      const double fbr = fbar[(size_t)A * PG.PN + max(pf, 0)];
      const double r0 = Ac.rho(m2), r1 = Ac.rho(m1), r2 = Ac.rho(f), r3 = Ac.rho(p1);
      const double e0 = Ac.e(m2), e1 = Ac.e(m1), e2 = Ac.e(f), e3 = Ac.e(p1);
      const double Wf = Ac.W(1, f), Wm = Ac.W(1, m1);
      const double fl = MF(A, f);
      double gg[4];
      // mass flux f_A = u_A rho*: rho at f - 2 .. f + 1
      const double fb = (pf >= 0) ? fbr : 0.0;
      upwind_grad(r0, r1, r2, r3, wv, gg);
#pragma unroll
      for (int j = 0; j < 4; ++j) g[j] = (fb != 0.0) ? fb * wv * gg[j] : 0.0;
      // energy flux g_A = f_A e*: e at f - 2 .. f + 1
      const double gb = (Wf - Wm) * ih;
      upwind_grad(e0, e1, e2, e3, wv, gg);
#pragma unroll
      for (int j = 0; j < 4; ++j) g[4 + j] = (gb != 0.0) ? gb * fl * gg[j] : 0.0;
      // conduction q = chi_f (T0 - Tm) ih with Tm at f - e_A, T0 at f (not on wall faces)
      if (G.chi_model != 0 && !(G.bc[A] == 1 && (f[A] == 0 || f[A] == G.n[A]))) {
        const double qb = (Wm - Wf) * ih;
        if (qb != 0.0) {
          const double Tm = eos_T<RAD>(G, r1, e1), T0 = eos_T<RAD>(G, r2, e2);
          double chm, ch0, dchm, dch0;
          if (G.chi_model == 1) {
            chm = ch0 = G.chi0;
            dchm = dch0 = 0.0;
          } else {
            const double pe = G.chi_exp;
            chm = G.chi0 * powr(Tm * G.chi_tref_inv, pe);
            ch0 = G.chi0 * powr(T0 * G.chi_tref_inv, pe);
            dchm = pe * chm / Tm;
            dch0 = pe * ch0 / T0;
          }
          const double chif = 0.5 * (chm + ch0);
          const double dT = T0 - Tm;
          const double qm = qb * (0.5 * dchm * dT - chif) * ih;  // times dT/dX of cell f - e_A
          const double q0 = qb * (0.5 * dch0 * dT + chif) * ih;  // times dT/dX of cell f
          if constexpr (RAD) {
            const Thermo tm = thermo<true>(G, r1, e1);
            const Thermo t0 = thermo<true>(G, r2, e2);
            g[1] += qm * tm.dTdr;
            g[2] += q0 * t0.dTdr;
            g[5] += qm * tm.dTde;
            g[6] += q0 * t0.dTde;
          } else {
            g[5] += qm * gm1;
            g[6] += q0 * gm1;
          }
        }
      }
    };
    double acc[2] = {0.0, 0.0};
    bscatter<ND, A, 2>(T, l, own, sC, coef, acc);
    rb += acc[0];
    eb += acc[1];
  }
  // Phi_AA: point q stands for the centre between faces q - e_A and q; u_A at q - 2 .. q + 1
  {
    auto coef = [&](const int* q, double* g) {
      SH(qm, q, A, -1);
      SH(qm2, q, A, -2);
      SH(qp1, q, A, 1);
      const double Wq = Ac.W(2 + A, q), Wqm = Ac.W(2 + A, qm);
      const double fm = MF(A, qm), f0 = MF(A, q);
      const double u0 = Ac.u(A, qm2), u1 = Ac.u(A, qm), u2 = Ac.u(A, q), u3 = Ac.u(A, qp1);
      const double Pb = (Wq - Wqm) * ih;
      const double m = 0.5 * (fm + f0);
      double gg[4];
      upwind_grad(u0, u1, u2, u3, m, gg);
#pragma unroll
      for (int j = 0; j < 4; ++j) g[j] = (Pb != 0.0) ? Pb * m * gg[j] : 0.0;
    };
    double acc[1] = {0.0};
    bscatter<ND, A, 1>(T, l, own, sC, coef, acc);
    ub[A] += acc[0];
  }
  // Phi_dA, d != A: the edge at point q carries u_d along A with the mass flux mean of f_A at
  // q - e_d and q; u_d at q - 2 .. q + 1 along A
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    if (d == A) continue;
    auto coef = [&](const int* q, double* g) {
      SH(qm, q, A, -1);
      SH(qd, q, d, -1);
      SH(qm2, q, A, -2);
      SH(qp1, q, A, 1);
      const double Wq = Ac.W(2 + d, q), Wqm = Ac.W(2 + d, qm);
      const double fd = MF(A, qd), f0 = MF(A, q);
      const double u0 = Ac.u(d, qm2), u1 = Ac.u(d, qm), u2 = Ac.u(d, q), u3 = Ac.u(d, qp1);
      const double Pb = (Wq - Wqm) * ih;
      const double m = 0.5 * (fd + f0);
      double gg[4];
      upwind_grad(u0, u1, u2, u3, m, gg);
#pragma unroll
      for (int j = 0; j < 4; ++j) g[j] = (Pb != 0.0) ? Pb * m * gg[j] : 0.0;
    };
    double acc[1] = {0.0};
    bscatter<ND, A, 1>(T, l, own, sC, coef, acc);
    ub[d] += acc[0];
  }
}

// terms local to the padded cell c: pressure in -p div u and in the momentum gradients,
// gravity, the cell's own mass flux (u_d times rho*), u_d in div u
template <int ND, bool RAD, class AC>
__device__ __forceinline__ void vjp_localB(const Grid& G, const PadGrid& PG, const AC& Ac, const int* c, int pl,
                                           const double* fbar, double& rb, double& eb, double* ub) {
  const double gm1 = G.gamma - 1.0;
  // all loads first (as in the scatter passes).  The terms are added unconditionally: a term
  // of weight zero adds an exact zero (its factors are finite), and the accumulators start at
  // +0 and so never hold -0, which is what adding +0 would change
  const double WE = Ac.W(1, c);
  const double rho0 = Ac.rho(c), e0 = Ac.e(c);
  double uc[3], ucp[3], Wc[3], Wcp[3], fb[3], rm2[3], rm1[3], rp1[3], em1[3], Wm[3];
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    SH(cp, c, d, 1);
    SH(m2, c, d, -2);
    SH(m1, c, d, -1);
    uc[d] = Ac.u(d, c);
    ucp[d] = Ac.u(d, cp);
    Wc[d] = Ac.W(2 + d, c);
    Wcp[d] = Ac.W(2 + d, cp);
    fb[d] = fbar[(size_t)d * PG.PN + pl];
    rm2[d] = Ac.rho(m2);
    rm1[d] = Ac.rho(m1);
    rp1[d] = Ac.rho(cp);
    em1[d] = Ac.e(m1);
    Wm[d] = Ac.W(1, m1);
  }
  double pbar = 0.0;
  {
    double D = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) D += (ucp[d] - uc[d]) * G.idx[d];
    pbar -= WE * D;
  }
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    pbar += (Wcp[d] - Wc[d]) * G.idx[d];
    rb += 0.5 * G.g[d] * (Wc[d] + Wcp[d]);
  }
  if constexpr (RAD) {
    const Thermo th = thermo<true>(G, rho0, e0);
    rb += pbar * th.dpdr;
    eb += pbar * th.dpde;
  } else if (pbar != 0.0) {
    rb += pbar * gm1 * e0;
    eb += pbar * gm1 * rho0;
  }
  const double p0 = eos_p<RAD>(G, rho0, e0);
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const double ih = G.idx[d];
    // the cell's own mass flux u_d rho*, the pressure gradients of the faces c and c + e_d
    ub[d] += fb[d] * upwind(rm2[d], rm1[d], rho0, rp1[d], uc[d]);
    ub[d] += WE * p0 * ih;
    ub[d] -= Wm[d] * eos_p<RAD>(G, rm1[d], em1[d]) * ih;
  }
}

template <int ND, bool RAD, class AC>
__device__ __forceinline__ void vjp_tileB(const Grid& G, const PadGrid& PG, const AC& Ac, const BTile<ND>& T,
                                          const double* mf, const double* fbar, double* xbar, double* sC) {
  const int t = threadIdx.x;
  const int l[3] = {t % bt<ND>(0), (t / bt<ND>(0)) % bt<ND>(1), t / (bt<ND>(0) * bt<ND>(1))};
  int c[3], pl = 0;
  bool own = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    c[d] = T.o[d] + l[d];
    if (d < ND) {
      own = own && (c[d] + 3 < PG.P[d]);
      pl += (c[d] + 3) * PG.pstride[d];
    }
  }
  double rb = 0.0, eb = 0.0, ub[3] = {0.0, 0.0, 0.0};
  vjp_axisB<ND, 0, RAD>(G, PG, Ac, T, l, own, mf, fbar, sC, rb, eb, ub);
  vjp_axisB<ND, 1, RAD>(G, PG, Ac, T, l, own, mf, fbar, sC, rb, eb, ub);
  if constexpr (ND == 3) vjp_axisB<ND, 2, RAD>(G, PG, Ac, T, l, own, mf, fbar, sC, rb, eb, ub);
  if (!own) return;
  vjp_localB<ND, RAD>(G, PG, Ac, c, pl, fbar, rb, eb, ub);
  xbar[pl] = rb;
  xbar[(size_t)PG.PN + pl] = eb;
#pragma unroll
  for (int d = 0; d < ND; ++d) xbar[(size_t)(2 + d) * PG.PN + pl] = ub[d];
}

template <int ND, bool RAD>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) k_vjp_stageB(Grid G, PadGrid PG, const double* X, const double* w,
                                                       double cR, const double* mf, const double* fbar,
                                                       double* xbar) {
  __shared__ double sC[8 * bfaces_max<ND>()];
  const BTile<ND> T = btile_setup<ND>(G, PG);
  if (T.interior) vjp_tileB<ND, RAD>(G, PG, Acc<ND, true>(G, X, w, cR), T, mf, fbar, xbar, sC);
  else vjp_tileB<ND, RAD>(G, PG, Acc<ND, false>(G, X, w, cR), T, mf, fbar, xbar, sC);
}

// ---- fold: interior adjoint = U part + sum of padded copies ------------------------------
// padded logical positions that hold a copy of stored index i on an axis, with signs
// padded logical positions that hold a copy of stored index i on an axis: slot 0 the index
// itself, slots 1 and 2 its images below and above the grid, with the sign of the copy (0: no
// copy in that slot)
__device__ __forceinline__ void preimages(int i, int n, int bc, bool normal, int* pos, double* sg) {
  if (bc == 0) {
    pos[0] = i;
    sg[0] = 1.0;
    pos[1] = i - n;
    sg[1] = (i - n >= -3) ? 1.0 : 0.0;
    pos[2] = i + n;
    sg[2] = (i + n <= n + 2) ? 1.0 : 0.0;
  } else if (!normal) {
    pos[0] = i;
    sg[0] = 1.0;
    pos[1] = -1 - i;
    sg[1] = (-1 - i >= -3) ? 1.0 : 0.0;
    pos[2] = 2 * n - 1 - i;
    sg[2] = (2 * n - 1 - i <= n + 2) ? 1.0 : 0.0;
  } else {
    pos[0] = i;
    sg[0] = (i >= 1) ? 1.0 : 0.0;
    pos[1] = -i;
    sg[1] = (i >= 1 && -i >= -3) ? -1.0 : 0.0;
    pos[2] = 2 * n - i;
    sg[2] = (i >= 1 && 2 * n - i <= n + 2) ? -1.0 : 0.0;
  }
}

template <int ND>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) k_vjp_fold(Grid G, PadGrid PG, const double* X, const double* w,
                                                     double cU, const double* xbar, int scaleR, double alpha2,
                                                     double* out) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (lin >= G.N) return;
  Pos P = make_pos<ND>(G, lin);
  const int N = G.N;
  double res[2 + ND];
  // U part: (dU/dX)^T (cU w) with U = (rho, rho e, rho_f u_d), rho_f the face mean
  {
    const double rho = X[lin], e = X[N + lin];
    double r0 = w[lin] + e * w[N + lin];
    double r1 = rho * w[N + lin];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      double s;
      int im = gidx<ND>(G, P, 0, shift(off0(), d, -1), &s);
      double rf = 0.5 * (X[im] + rho);
      double wd = w[(2 + d) * N + lin];
      double ud = X[(2 + d) * N + lin];
      res[2 + d] = cU * rf * wd;
      r0 += 0.5 * ud * wd;
      if (G.bc[d] == 1 && P.c[d] == 0) r0 += 0.5 * ud * wd;  // mirror ghost rho[-1] = rho[0]
      // face c + e_d reads rho[c] as its lower cell
      bool has_up = !(G.bc[d] == 1 && P.c[d] == G.n[d] - 1);
      if (has_up) {
        int ip = (P.c[d] == G.n[d] - 1) ? lin - (G.n[d] - 1) * G.stride[d] : lin + G.stride[d];
        r0 += 0.5 * X[(2 + d) * N + ip] * w[(2 + d) * N + ip];
      }
    }
    res[0] = cU * r0;
    res[1] = cU * r1;
  }
  // R part: sum over padded copies (a cell at least 4 cells from both ends of every axis has
  // no image in the padded grid, only itself with sign +1, whatever the axis's boundary)
  bool inner = true;
#pragma unroll
  for (int d = 0; d < ND; ++d) inner = inner && P.c[d] >= 4 && P.c[d] <= G.n[d] - 4;
  if (inner) {
    int pl = (P.c[0] + 3) + (P.c[1] + (ND >= 2 ? 3 : 0)) * PG.pstride[1];
    if (ND == 3) pl += (P.c[2] + 3) * PG.pstride[2];
#pragma unroll
    for (int var = 0; var < 2 + ND; ++var) res[var] += xbar[(size_t)var * PG.PN + pl];
  }
#pragma unroll
  for (int var = 0; var < 2 + ND; ++var) {
    if (inner) break;
    int pos[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double sg[3][3] = {{1.0, 0.0, 0.0}, {1.0, 0.0, 0.0}, {1.0, 0.0, 0.0}};
#pragma unroll
    for (int d = 0; d < ND; ++d) preimages(P.c[d], G.n[d], G.bc[d], var == 2 + d, pos[d], sg[d]);
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          const double sgn = sg[0][a] * sg[1][b] * sg[2][cc];
          if (sgn == 0.0) continue;  // no copy there (the position may lie off the padded grid)
          int pl = (pos[0][a] + 3) + (pos[1][b] + (ND >= 2 ? 3 : 0)) * PG.pstride[1];
          if (ND == 3) pl += (pos[2][cc] + 3) * PG.pstride[2];
          acc += sgn * xbar[(size_t)var * PG.PN + pl];
        }
    res[var] += acc;
  }
  if (scaleR) {
    const double e0 = X[N + lin];
    const double cs0 = sound_speed_rt(G, X[lin], e0);
    res[0] *= X[lin];
    res[1] *= e0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      double s;
      int im = gidx<ND>(G, P, 1, shift(off0(), d, -1), &s);
      double csf = 0.5 * (sound_speed_rt(G, X[im], X[N + im]) + cs0);
      res[2 + d] *= fmax(fabs(X[(2 + d) * N + lin]), alpha2 * csf);
    }
  }
#pragma unroll
  for (int v = 0; v < 2 + ND; ++v) out[v * N + lin] = res[v];
}

// ---- transposed physics-based preconditioner ---------------------------------------------
// The forward map r -> z is: F_V = dV/dU r; dp = A_p^-1 (F_p/(Gamma1 p)); de from the
// identity (sound) or dT = A_T^-1 (rho F_e + (dp/dt - F_p)/Gamma1), de = c_v dT (thermal);
// du = dt (F_u - grad dp / rho_f); drho from the linearised EOS.  Its transpose applies the
// transposed pointwise maps in reverse order around the same (symmetric) solves.

// adjoint input w of one cell (w = v / R(X) when scaled) and the EOS factors
template <int ND>
struct CellT {
  double rho, e, dpdr, dpde, wr, we;
};

template <int ND>
__device__ __forceinline__ double rscale_u(const Grid& G, const Pos& P, const double* X, int d,
                                           double alpha2) {
  double s;
  int im = gidx<ND>(G, P, 1, shift(off0(), d, -1), &s);
  double csf = 0.5 * (sound_speed_rt(G, X[im], X[G.N + im]) + sound_speed_rt(G, X[P.lin], X[G.N + P.lin]));
  return fmax(fabs(X[(2 + d) * G.N + P.lin]), alpha2 * csf);
}

// w_d at face lin of axis d (divided by R_u there when scaled)
template <int ND>
__device__ __forceinline__ double w_face(const Grid& G, const double* X, const double* v, int scaled,
                                         double alpha2, int d, int lin) {
  double wv = v[(2 + d) * G.N + lin];
  if (scaled) {
    Pos Q = make_pos<ND>(G, lin);
    wv /= rscale_u<ND>(G, Q, X, d, alpha2);
  }
  return wv;
}

// transposed face gradient: sum over the faces of c of a_d[f] d(grad dp)[f]/d dp[c] with
// grad dp[f] = (dp[f] - dp[f-1])/(rho_f dx_d), zero on wall faces
template <int ND>
__device__ __forceinline__ double gradT(const Grid& G, const Pos& P, const double* X, const double* v,
                                        int scaled, double alpha2) {
  double acc = 0.0;
  const int N = G.N;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    double s;
    // own face c: + a[c]/(rho_f[c] dx)
    if (!(G.bc[d] == 1 && P.c[d] == 0)) {
      int im = gidx<ND>(G, P, 0, shift(off0(), d, -1), &s);
      double rf = 0.5 * (X[im] + X[P.lin]);
      acc += w_face<ND>(G, X, v, scaled, alpha2, d, P.lin) / (rf * G.dx[d]);
    }
    // upper face c + e_d: - a[c+e]/(rho_f[c+e] dx)
    bool top = (P.c[d] == G.n[d] - 1);
    if (!(G.bc[d] == 1 && top)) {
      int ip = top ? P.lin - (G.n[d] - 1) * G.stride[d] : P.lin + G.stride[d];
      double rf = 0.5 * (X[P.lin] + X[ip]);
      if (!(G.bc[d] == 1 && top)) acc -= w_face<ND>(G, X, v, scaled, alpha2, d, ip) / (rf * G.dx[d]);
    }
    (void)N;
  }
  return acc;
}

template <int ND>
__global__ void __launch_bounds__(kBlock) k_pbpT_in(Grid G, const double* X, const double* v, int scaled,
                                                    double alpha2, double dt, int thermal, double* rhs_p,
                                                    double* rhs_T) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (lin >= G.N) return;
  Pos P = make_pos<ND>(G, lin);
  const double gm1 = G.gamma - 1.0;
  double rho = X[lin], e = X[G.N + lin];
  double wr = v[lin], we = v[G.N + lin];
  if (scaled) {
    wr /= rho;
    we /= e;
  }
  const Thermo th = thermo_rt(G, rho, e);
  const double dpdr = th.dpdr, dpde = th.dpde;
  double dp_b = wr / dpdr;
  double de_b = we - dpde / dpdr * wr;
  dp_b -= dt * gradT<ND>(G, P, X, v, scaled, alpha2);
  if (!thermal) {
    rhs_p[lin] = dp_b + de_b / (th.G1 * rho);
  } else {
    rhs_p[lin] = dp_b;  // completed by k_pbpT_mid after the thermal solve
    rhs_T[lin] = G.a_rad == 0.0 ? de_b / gm1 : th.cv * de_b;  // c_v de_b
  }
}

__global__ void __launch_bounds__(kBlock) k_pbpT_mid(Grid G, const double* X, double dt, const double* t,
                                                     double* rhs_p) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (lin >= G.N) return;
  const double g1 = G.a_rad == 0.0 ? G.gamma : thermo<true>(G, X[lin], X[G.N + lin]).G1;
  rhs_p[lin] += t[lin] / (g1 * dt);
}

template <int ND>
__global__ void __launch_bounds__(kBlock) k_pbpT_out(Grid G, const double* X, const double* v, int scaled,
                                                     double alpha2, double dt, const double* sp,
                                                     const double* t, int schur, double zs, double* z) {
  int lin = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (lin >= G.N) return;
  Pos P = make_pos<ND>(G, lin);
  const int N = G.N;
  double rho = X[lin], e = X[N + lin];
  double wr = v[lin], we = v[N + lin];
  if (scaled) {
    wr /= rho;
    we /= e;
  }
  const Thermo th = thermo_rt(G, rho, e);
  const double dpdr = th.dpdr, dpde = th.dpde;
  double de_b = we - dpde / dpdr * wr;
  double Fe_b, Fp_b;
  if (t) {
    Fe_b = rho * t[lin];
    Fp_b = -t[lin] / th.G1;
  } else {
    Fe_b = dt * de_b;
    Fp_b = -dt * de_b / (th.G1 * rho);
  }
  Fp_b += sp[lin] / (th.G1 * th.p);
  double r0 = (dpdr - (e / rho) * dpde) * Fp_b - (e / rho) * Fe_b;
  double r1 = (dpde / rho) * Fp_b + Fe_b / rho;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    double s;
    int im = gidx<ND>(G, P, 0, shift(off0(), d, -1), &s);
    double rf = 0.5 * (X[im] + rho);
    double Fu_b = dt * w_face<ND>(G, X, v, scaled, alpha2, d, lin);
    // schur: the pressure right-hand side's -dt div F_u, transposed (not on wall faces)
    if (schur && !(G.bc[d] == 1 && P.c[d] == 0)) Fu_b -= dt * (sp[im] - sp[lin]) * G.idx[d];
    z[(2 + d) * N + lin] = zs * (Fu_b / rf);
    // the F_u row of face f reads rbar = (r_rho[f-1] + r_rho[f])/2 with coefficient -u/rho_f
    double a0 = -X[(2 + d) * N + lin] * Fu_b / rf;
    r0 += 0.5 * a0;
    if (G.bc[d] == 1 && P.c[d] == 0) r0 += 0.5 * a0;  // mirror ghost r_rho[-1] = r_rho[0]
    bool top = (P.c[d] == G.n[d] - 1);
    if (!(G.bc[d] == 1 && top)) {
      int ip = top ? lin - (G.n[d] - 1) * G.stride[d] : lin + G.stride[d];
      double rfp = 0.5 * (rho + X[ip]);
      double Fu_bp = dt * w_face<ND>(G, X, v, scaled, alpha2, d, ip);
      if (schur) Fu_bp -= dt * (sp[lin] - sp[ip]) * G.idx[d];
      r0 += 0.5 * (-X[(2 + d) * N + ip] * Fu_bp / rfp);
    }
  }
  z[lin] = zs * r0;
  z[N + lin] = zs * r1;
}

void launch_pbpT_in(const Grid& G, const double* X, const double* v, int scaled, double alpha2,
                    double dt, int thermal, double* rhs_p, double* rhs_T, hipStream_t s) {
  dim3 gr((G.N + kBlock - 1) / kBlock);
  if (G.nd == 2) k_pbpT_in<2><<<gr, kBlock, 0, s>>>(G, X, v, scaled, alpha2, dt, thermal, rhs_p, rhs_T);
  else k_pbpT_in<3><<<gr, kBlock, 0, s>>>(G, X, v, scaled, alpha2, dt, thermal, rhs_p, rhs_T);
}
void launch_pbpT_mid(const Grid& G, const double* X, double dt, const double* t, double* rhs_p,
                     hipStream_t s) {
  dim3 gr((G.N + kBlock - 1) / kBlock);
  k_pbpT_mid<<<gr, kBlock, 0, s>>>(G, X, dt, t, rhs_p);
}
void launch_pbpT_out(const Grid& G, const double* X, const double* v, int scaled, double alpha2,
                     double dt, const double* sp, const double* t, int schur, double zscale, double* z,
                     hipStream_t s) {
  dim3 gr((G.N + kBlock - 1) / kBlock);
  if (G.nd == 2) k_pbpT_out<2><<<gr, kBlock, 0, s>>>(G, X, v, scaled, alpha2, dt, sp, t, schur, zscale, z);
  else k_pbpT_out<3><<<gr, kBlock, 0, s>>>(G, X, v, scaled, alpha2, dt, sp, t, schur, zscale, z);
}

size_t vjp_scratch_doubles(const Grid& G) {
  PadGrid PG = make_pad(G);
  return (size_t)PG.PN * (G.nd + 2 + G.nd + G.nd);
}

void launch_vjp(const Grid& G, const double* X, const double* w, double cU, double cR, double* scratch,
                int scaleR, double alpha2, double* out, hipStream_t s) {
  PadGrid PG = make_pad(G);
  double* fbar = scratch;
  double* xbar = scratch + (size_t)G.nd * PG.PN;
  double* mf = xbar + (size_t)(2 + G.nd) * PG.PN;
  dim3 gp((PG.PN + kBlock - 1) / kBlock), gc((G.N + kBlock - 1) / kBlock), bl(kBlock);
  const double nv = 2 + G.nd;
  {
    const double by = 8.0 * (3.0 * G.N + G.nd * (double)PG.PN);
    if (G.nd == 2) launch_k(KF_VJP_A, by, k_vjp_flux<2>, gp, bl, 0, s, G, PG, X, mf);
    else launch_k(KF_VJP_A, by, k_vjp_flux<3>, gp, bl, 0, s, G, PG, X, mf);
  }
  const double* mfc = mf;
  {
    const double by = 8.0 * (2 * nv * G.N + 2 * G.nd * (double)PG.PN);
    const dim3 ga(G.nd == 2 ? btile_blocks<2>(PG) : btile_blocks<3>(PG));
    if (G.nd == 2) launch_k(KF_VJP_A, by, k_vjp_stageA<2>, ga, bl, 0, s, G, PG, X, w, cR, mfc, fbar);
    else launch_k(KF_VJP_A, by, k_vjp_stageA<3>, ga, bl, 0, s, G, PG, X, w, cR, mfc, fbar);
  }
  {
    const double by = 8.0 * (2 * nv * G.N + (2 * G.nd + nv) * (double)PG.PN);
    const double* fb = fbar;
    const bool rad = G.a_rad != 0.0;
    const dim3 gb(G.nd == 2 ? btile_blocks<2>(PG) : btile_blocks<3>(PG));
    if (G.nd == 2)
      launch_k(KF_VJP_B, by, rad ? k_vjp_stageB<2, true> : k_vjp_stageB<2, false>, gb, bl, 0, s, G, PG, X, w,
               cR, mfc, fb, xbar);
    else
      launch_k(KF_VJP_B, by, rad ? k_vjp_stageB<3, true> : k_vjp_stageB<3, false>, gb, bl, 0, s, G, PG, X, w,
               cR, mfc, fb, xbar);
  }
  {
    const double by = 8.0 * (3 * nv * G.N + nv * (double)PG.PN);
    const double* xb = xbar;
    if (G.nd == 2)
      launch_k(KF_VJP_FOLD, by, k_vjp_fold<2>, gc, bl, 0, s, G, PG, X, w, cU, xb, scaleR, alpha2, out);
    else
      launch_k(KF_VJP_FOLD, by, k_vjp_fold<3>, gc, bl, 0, s, G, PG, X, w, cU, xb, scaleR, alpha2, out);
  }
}

}  // namespace jfnk
