// Device helpers shared by the forward and adjoint kernels of the HOPE
// right-hand side: fast reciprocal/root, LMARS, sources, and the
// reconstruction building blocks (TPP (3.14), genuine 2D WENO (3.16)-(3.25)).
#pragma once
#include <hip/hip_runtime.h>

#include "hope_internal.hpp"

namespace hope {

typedef const __attribute__((address_space(4))) double* cdp;
typedef const __attribute__((address_space(4))) int32_t* cip;

// The chip dispatches workgroup b to L2 domain (XCD) b % 8.  xcd_block(b, nb)
// (nb a multiple of 8) gives each domain a contiguous range of logical
// blocks; it is a bijection of [0, nb).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int nb) { return (b % kXcds) * (nb / kXcds) + b / kXcds; }

// ---------------------------------------------------------------------------
// Arithmetic helpers
// ---------------------------------------------------------------------------
// reciprocal: the hardware estimate (relative error below 2^-24 on gfx950)
// refined by one Newton-Raphson step, which squares that error: at most 11
// units in the last place over 4M arguments spanning 2^-40..2^40, far below
// the rounding already carried by the sums these values divide
__device__ __forceinline__ double rcp(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

// square root: one Goldschmidt step from the hardware reciprocal square root
// (relative error below 2^-24) and a final Newton correction of the root,
// which together give the correctly rounded root on every one of 4M
// arguments spanning 2^-40..2^40
__device__ __forceinline__ double sqrt_g(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  return fma(d, h, g);
}

// LMARS flux (3.30)-(3.38) with upwind term |m|(q_R - q_L); dir 0 = x, 1 = y.
// sqx = sqrt(1 + X^2), sqy = sqrt(1 + Y^2) come from tables, ia = 1/a.
// TOPO: bottom topography (2.13); q holds the layer's own sqrtG phi and
// sps = sqrtG phi_s at the point, so the pressure uses phi_t* = phi* + phi_s
// (both sides share phi_s, so the height jump of (3.32) is that of phi_t).
template <bool TOPO = false>
__device__ __forceinline__ void lmars(const double* qL, const double* qR, double X, double Y, double sqx,
                                      double sqy, int dir, double ia, double* F, double sps = 0.0) {
  const double ox = sqx * sqx, oy = sqy * sqy;
  const double d2 = fma(X, X, oy);
  const double dl = sqrt_g(d2);
  const double idl = rcp(dl);
  const double isg = d2 * dl * ia * ia * rcp(ox * oy);            // 1/sqrtG, (2.8)
  const double sgii = dl * ia * rcp(dir == 0 ? sqx : sqy);        // sqrt(G^ii), (2.6)
  const int iv = 1 + dir;
  const double phiL = qL[0] * isg, phiR = qR[0] * isg;
  const double upL = qL[iv] * rcp(qL[0] * sgii);                   // (3.31)
  const double upR = qR[iv] * rcp(qR[0] * sgii);
  const double c = 0.5 * (sqrt_g(phiL) + sqrt_g(phiR));           // (3.34)-(3.35)
  const double ms = 0.5 * (upL + upR - (phiR - phiL) * rcp(c));   // (3.32)
  double ps = 0.5 * (phiL + phiR - c * (upR - upL));              // (3.33)
  if constexpr (TOPO) ps = fma(sps, isg, ps);                     // phi_t* = phi* + phi_s
  const double mm = ms * sgii;                                    // (3.36)
  const double am = fabs(mm);
#pragma unroll
  for (int v = 0; v < 3; ++v) F[v] = 0.5 * (mm * (qL[v] + qR[v]) - am * (qR[v] - qL[v]));   // (3.37)
  const double pr = 0.5 * ps * ps * idl;                          // (3.38): sqrtG G^ij = (..)/delta
  if (dir == 0) {
    F[1] = fma(pr, oy, F[1]);
    F[2] = fma(pr, X * Y, F[2]);
  } else {
    F[1] = fma(pr, X * Y, F[1]);
    F[2] = fma(pr, ox, F[2]);
  }
}

// Metric (2.2) and Coriolis (2.3) sources at one point; Lc = c0 + cX X + cY Y
// so that f*delta = 2 Omega Lc.
__device__ __forceinline__ void sources(double Q0, double Q1, double Q2, double X, double Y, double Lc,
                                        double omega2, double& s1, double& s2) {
  const double X2 = X * X, Y2 = Y * Y;
  const double id2 = rcp(1.0 + X2 + Y2);
  const double iq = 2.0 * rcp(Q0);
  const double m1 = iq * (Y * (1.0 + Y2) * Q1 * Q2 - X * Y2 * Q1 * Q1);
  const double m2 = iq * (X * (1.0 + X2) * Q1 * Q2 - X2 * Y * Q2 * Q2);
  const double f = omega2 * Lc;
  const double c1 = f * ((1.0 + Y2) * Q2 - X * Y * Q1);
  const double c2 = f * (X * Y * Q2 - (1.0 + X2) * Q1);
  s1 = (m1 + c1) * id2;
  s2 = (m2 + c2) * id2;
}

// sqrtG phi_s of the topography tables at point h of the side sd (0 left,
// 1 right, 2 bottom, 3 top) of cell (i, j) of panel p
template <int M>
__device__ __forceinline__ double topo_cell_side(const TopoDev& tp, int n, int p, int i, int j, int sd, int h) {
  if (sd < 2) return tp.sx[(((size_t)p * n + j) * (n + 1) + i + sd) * M + h];
  return tp.sy[(((size_t)p * (n + 1) + j + (sd - 2)) * n + i) * M + h];
}

// the same at point h of a panel's boundary side idx = (panel*4 + side)*n + t
template <int M>
__device__ __forceinline__ double topo_side_point(const TopoDev& tp, int n, int idx, int h) {
  const int p = idx / (4 * n), side = (idx / n) % 4, t = idx % n;
  if (side < 2) return tp.sx[(((size_t)p * n + t) * (n + 1) + (side ? n : 0)) * M + h];
  return tp.sy[(((size_t)p * (n + 1) + (side == 3 ? n : 0)) * n + t) * M + h];
}

// Bottom-topography source psi_B (2.14) at one point.  T = sqrtG phi_t,
// (Txi, Teta) its derivatives in the unit-cell coordinates of the
// reconstruction polynomial, sps = sqrtG phi_s; invd = 1/Delta, ia = 1/a.
// With D_j = dT/dx^j - T d(ln sqrtG)/dx^j, d(ln sqrtG)/dx = X (2Y^2 - X^2 - 1)
// / delta^2 (from (2.8)), d(phi_t)/dx^j = D_j / sqrtG, and
// psi_B^i = sps G^ij D_j / sqrtG = sps delta^5 / (a^4 ox^2 oy^2) times
// (oy D_x + X Y D_y, X Y D_x + ox D_y), ox = 1 + X^2, oy = 1 + Y^2.
__device__ __forceinline__ double psi_b_scale(double X, double Y, double sps, double ia, double& ox, double& oy,
                                              double& ex, double& ey) {
  const double X2 = X * X, Y2 = Y * Y;
  ox = 1.0 + X2;
  oy = 1.0 + Y2;
  const double d2 = ox + Y2;
  const double id2 = rcp(d2);
  ex = X * (2.0 * Y2 - X2 - 1.0) * id2;
  ey = Y * (2.0 * X2 - Y2 - 1.0) * id2;
  const double ia2 = ia * ia;
  const double oo = rcp(ox * oy);
  return sps * d2 * d2 * sqrt_g(d2) * ia2 * ia2 * oo * oo;
}

__device__ __forceinline__ void psi_b(double T, double Txi, double Teta, double X, double Y, double sps, double invd,
                                      double ia, double& b1, double& b2) {
  double ox, oy, ex, ey;
  const double c = psi_b_scale(X, Y, sps, ia, ox, oy, ex, ey);
  const double Dx = fma(Txi, invd, -T * ex), Dy = fma(Teta, invd, -T * ey);
  const double xy = X * Y;
  b1 = c * fma(oy, Dx, xy * Dy);
  b2 = c * fma(xy, Dx, ox * Dy);
}

// reverse mode of psi_b: given (b1b, b2b) = dL/d(b1, b2), the cotangents of
// T, Txi and Teta
__device__ __forceinline__ void psi_b_adj(double X, double Y, double sps, double invd, double ia, double b1b,
                                          double b2b, double& Tb, double& Txib, double& Tetab) {
  double ox, oy, ex, ey;
  const double c = psi_b_scale(X, Y, sps, ia, ox, oy, ex, ey);
  const double xy = X * Y;
  const double Dxb = c * fma(oy, b1b, xy * b2b), Dyb = c * fma(xy, b1b, ox * b2b);
  Txib = Dxb * invd;
  Tetab = Dyb * invd;
  Tb = -(Dxb * ex + Dyb * ey);
}

// ---------------------------------------------------------------------------
// Reconstruction of one cell from a stencil accessor at(dy, dx).  Axis
// coordinates: 0 -> -1/2, 1 -> +1/2, 2+h -> Gauss node h.  Point numbering of
// one cell: x-edge left (h), x-edge right (h), y-edge bottom (h), y-edge top
// (h), CQP (v outer, h inner).
// ---------------------------------------------------------------------------
template <int K, bool W, int M>
struct Cfg {
  static constexpr int R = (K - 1) / 2;
  static constexpr int L = (K + 1) / 2;     // sub-stencil width (WENO)
  static constexpr int S = L * L;
  static constexpr int NA = 2 + M;
  static constexpr int NR = 2 * R + 1;
  static constexpr int XR = W ? L * NR : NR;
  static constexpr TabOffsets O = tab_offsets(K, W, M, 0);
};

// smoothness indicators -> kappa_j = 1 + tau/(beta_j + eps) of one variable,
// (3.23)-(3.25); out(j, kappa_j)
template <int K, bool W, int M, typename TP, typename At, typename Out>
__device__ __forceinline__ void weno_kappa(TP tab, double eps, At at, Out out) {
  using C = Cfg<K, W, M>;
  constexpr int L = C::L, S = C::S, NR = C::NR, R = C::R;
  TP V = tab + C::O.V, lam = tab + C::O.lam;
  double beta[S];
#pragma unroll
  for (int sx = 0; sx < L; ++sx) {
    double tr[NR][L];
#pragma unroll
    for (int row = 0; row < NR; ++row)
#pragma unroll
      for (int al = 0; al < L; ++al) {
        double s = 0;
#pragma unroll
        for (int a = 0; a < L; ++a) s = fma(V[(sx * L + al) * L + a], at(row - R, sx - (L - 1) + a), s);
        tr[row][al] = s;
      }
#pragma unroll
    for (int sy = 0; sy < L; ++sy) {
      double b = 0;
#pragma unroll
      for (int be = 0; be < L; ++be)
#pragma unroll
        for (int al = 0; al < L; ++al) {
          if (al == 0 && be == 0) continue;
          double c = 0;
#pragma unroll
          for (int bb = 0; bb < L; ++bb) c = fma(V[(sy * L + be) * L + bb], tr[sy + bb][al], c);
          b = fma(lam[be * L + al] * c, c, b);
        }
      beta[sy * L + sx] = b;
    }
  }
  double tau = 0;
#pragma unroll
  for (int a = 0; a < S; ++a)
#pragma unroll
    for (int b = a + 1; b < S; ++b) tau += fabs(beta[a] - beta[b]);
  tau *= 2.0 / (S * (S + 1));
#pragma unroll
  for (int j = 0; j < S; ++j) out(j, fma(tau, rcp(beta[j] + eps), 1.0));
}

// x-pass at axis px: TPP: xr[row]; WENO: xr[sx*NR + row]
template <int K, bool W, int M, typename TP, typename At>
__device__ __forceinline__ void xpass(TP tab, int px, At at, double* xr) {
  using C = Cfg<K, W, M>;
  constexpr int L = C::L, NR = C::NR, R = C::R, NA = C::NA;
  if constexpr (!W) {
    TP wc = tab + C::O.wc;
#pragma unroll
    for (int row = 0; row < NR; ++row) {
      double s = 0;
#pragma unroll
      for (int a = 0; a < K; ++a) s = fma(wc[px * K + a], at(row - R, a - R), s);
      xr[row] = s;
    }
  } else {
    TP wsub = tab + C::O.wsub;
#pragma unroll
    for (int sx = 0; sx < L; ++sx)
#pragma unroll
      for (int row = 0; row < NR; ++row) {
        double s = 0;
#pragma unroll
        for (int a = 0; a < L; ++a) s = fma(wsub[(sx * NA + px) * L + a], at(row - R, sx - (L - 1) + a), s);
        xr[sx * NR + row] = s;
      }
  }
}

// value at axis py from the x-pass; pt = point number; kap(j) gives kappa_j
template <int K, bool W, int M, typename TP, typename Kap>
__device__ __forceinline__ double point(TP tab, int py, int pt, const double* xr, Kap kap) {
  using C = Cfg<K, W, M>;
  constexpr int L = C::L, S = C::S, NR = C::NR, NA = C::NA;
  if constexpr (!W) {
    TP wc = tab + C::O.wc;
    double s = 0;
#pragma unroll
    for (int b = 0; b < K; ++b) s = fma(wc[py * K + b], xr[b], s);
    return s;
  } else {
    TP wsub = tab + C::O.wsub, gp = tab + C::O.gp, gm = tab + C::O.gm;
    double ap = 0, dp = 0, am = 0, dm = 0;
#pragma unroll
    for (int sy = 0; sy < L; ++sy)
#pragma unroll
      for (int sx = 0; sx < L; ++sx) {
        double pv = 0;
#pragma unroll
        for (int b = 0; b < L; ++b) pv = fma(wsub[(sy * NA + py) * L + b], xr[sx * NR + sy + b], pv);
        const int j = sy * L + sx;
        const double kj = kap(j);
        const double tk = kj * pv;
        ap = fma(gp[pt * S + j], tk, ap);
        am = fma(gm[pt * S + j], tk, am);
        dp = fma(gp[pt * S + j], kj, dp);
        dm = fma(gm[pt * S + j], kj, dm);
      }
    // (3.20)-(3.22): sigma+ sum w+ p - sigma- sum w- p, w = alpha / sum alpha
    return (tab[C::O.sp + pt] * ap * dm - tab[C::O.sm + pt] * am * dp) * rcp(dp * dm);
  }
}


// ---------------------------------------------------------------------------
// Genuine 2D WENO by columns.  The linear weights of a point factor as
// gamma_j = d_sy(py) d_sx(px) (tensor product of the 1D linear weights), and
// the split (3.20) gives gamma+- = (theta |gamma| +- gamma) / 2, so with
//   B = sum_j gamma_j kappa_j p_j,  A = sum_j |gamma_j| kappa_j p_j,
//   D = sum_j gamma_j kappa_j,      C = sum_j |gamma_j| kappa_j
// the value (3.21) is sigma+ (theta A + B)/(theta C + D)
//                     - sigma- (theta A - B)/(theta C - D),
// and where every gamma of the point is positive (A = B, C = D) it is B / D.
// The sums over the sub-stencil columns sx are shared by all points of one x
// axis point px: with the x-pass xr (sub-stencil sx, stencil row) and
//   Z[sy][b] = sum_sx d_sx kappa_(sy,sx) xr[sx][sy+b],  E[sy] = sum_sx d_sx kappa_(sy,sx)
// a point needs only B = sum_sy d_sy(py) sum_b w_(sy,b)(py) Z[sy][b] and
// D = sum_sy d_sy(py) E[sy] (and their |d| versions).
// ---------------------------------------------------------------------------
template <int K, int M>
struct WCol {
  static constexpr int L = (K + 1) / 2;
  double E[L], Z[L][L];       // with d_sx
  double Ea[L], Za[L][L];     // with |d_sx| (axis points of mixed sign only)
};

// column sums of x axis point px from its x-pass xr and the weights kappa
template <int K, bool W, int M, typename TP, typename Kap>
__device__ __forceinline__ void wcol(TP tab, int px, const double* xr, Kap kap, WCol<K, M>& c) {
  using C = Cfg<K, W, M>;
  constexpr int L = C::L, NR = C::NR;
  TP d1 = tab + C::O.d1;
  const bool mixed = weno_mixed_axis(K, M, px);
#pragma unroll
  for (int sy = 0; sy < L; ++sy) {
    double e[L];
    double E = 0.0;
#pragma unroll
    for (int sx = 0; sx < L; ++sx) {
      e[sx] = d1[px * L + sx] * kap(sy * L + sx);
      E += e[sx];
    }
    c.E[sy] = E;
#pragma unroll
    for (int b = 0; b < L; ++b) {
      double z = 0.0;
#pragma unroll
      for (int sx = 0; sx < L; ++sx) z = fma(e[sx], xr[sx * NR + sy + b], z);
      c.Z[sy][b] = z;
    }
    if (mixed) {
      double Ea = 0.0;
#pragma unroll
      for (int sx = 0; sx < L; ++sx) {
        e[sx] = fabs(d1[px * L + sx]) * kap(sy * L + sx);
        Ea += e[sx];
      }
      c.Ea[sy] = Ea;
#pragma unroll
      for (int b = 0; b < L; ++b) {
        double z = 0.0;
#pragma unroll
        for (int sx = 0; sx < L; ++sx) z = fma(e[sx], xr[sx * NR + sy + b], z);
        c.Za[sy][b] = z;
      }
    }
  }
}

// value at y axis point py (point number pt) of the column px prepared by wcol
template <int K, bool W, int M, typename TP>
__device__ __forceinline__ double wpoint(TP tab, int px, int py, int pt, const WCol<K, M>& c) {
  using C = Cfg<K, W, M>;
  constexpr int L = C::L, NA = C::NA;
  TP wsub = tab + C::O.wsub, d1 = tab + C::O.d1;
  const bool xm = weno_mixed_axis(K, M, px), ym = weno_mixed_axis(K, M, py);
  double B = 0.0, D = 0.0, A = 0.0, Cs = 0.0;
#pragma unroll
  for (int sy = 0; sy < L; ++sy) {
    double T = 0.0;
#pragma unroll
    for (int b = 0; b < L; ++b) T = fma(wsub[(sy * NA + py) * L + b], c.Z[sy][b], T);
    const double dy = d1[py * L + sy];
    B = fma(dy, T, B);
    D = fma(dy, c.E[sy], D);
    if (xm) {
      double Ta = 0.0;
#pragma unroll
      for (int b = 0; b < L; ++b) Ta = fma(wsub[(sy * NA + py) * L + b], c.Za[sy][b], Ta);
      A = fma(fabs(dy), Ta, A);
      Cs = fma(fabs(dy), c.Ea[sy], Cs);
    } else if (ym) {
      A = fma(fabs(dy), T, A);
      Cs = fma(fabs(dy), c.E[sy], Cs);
    }
  }
  if (!xm && !ym) return B * rcp(D);
  const double th = tab[C::O.theta];
  const double np = fma(th, A, B), dp = fma(th, Cs, D), nm = fma(th, A, -B), dm = fma(th, Cs, -D);
  return (tab[C::O.sp + pt] * np * dm - tab[C::O.sm + pt] * nm * dp) * rcp(dp * dm);
}

}  // namespace hope
