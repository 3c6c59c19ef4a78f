// HIP kernels (gfx950, FP64) of the HOPE right-hand side.
//
//  k_fill_halo     ghost cells g = G q (appendix (7.12)); 16 lanes per ghost row
//  k_edge_traces   at every panel-edge Gauss point, the neighbour panel's own
//                  trace, converted into this panel's variables (3.26)-(3.29)
//  k_stage         fused reconstruction (TPP (3.14) or genuine 2D WENO
//                  (3.16)-(3.25)), LMARS (3.30)-(3.38), Gauss quadrature of the
//                  fluxes (3.5) and sources (2.2)-(2.3), (3.6), the tendency
//                  (3.1) and an optional Runge-Kutta combination
//
// k_stage marches: one wavefront owns a strip of up to 62 interior columns of
// one panel (lanes 1..62; lanes 0 and 63 are the strip's ring columns) and a
// segment of rows, walking up the rows.  At each row every lane reconstructs
// its cell; the flux through the left edge of lane L takes the left state
// from lane L-1 by a cross-lane shuffle, and the flux through the bottom edge
// takes the top trace of the row below, which the lane kept in registers from
// the previous step.  No trace ever goes to memory.
#include <hip/hip_runtime.h>

#include "hope_internal.hpp"

namespace hope {

// Constant-address-space view of the grid tables: the tables never change
// while a kernel runs, and loads through this address space with uniform
// addresses become scalar loads into SGPRs instead of per-lane vector loads.
typedef const __attribute__((address_space(4))) double* cdp;
typedef const __attribute__((address_space(4))) int32_t* cip;

struct CTab {
  cdp wc, wsub, gp, gm, sp, sm, V, lam, Xe, Xg, sqe, sqg, gw, fcoef, bt_conv;
  cip bt_cell, bt_side, bt_rev;
  double radius, omega2, eps, inv_delta;
  int n, P, r, m;
  __device__ explicit CTab(const DevTables& d)
      : wc((cdp)d.wc), wsub((cdp)d.wsub), gp((cdp)d.gp), gm((cdp)d.gm), sp((cdp)d.sp), sm((cdp)d.sm),
        V((cdp)d.V), lam((cdp)d.lam), Xe((cdp)d.Xe), Xg((cdp)d.Xg), sqe((cdp)d.sqe), sqg((cdp)d.sqg),
        gw((cdp)d.gw), fcoef((cdp)d.fcoef), bt_conv((cdp)d.bt_conv), bt_cell((cip)d.bt_cell),
        bt_side((cip)d.bt_side), bt_rev((cip)d.bt_rev), radius(d.radius), omega2(d.omega2), eps(d.eps),
        inv_delta(d.inv_delta), n(d.n), P(d.P), r(d.r), m(d.m) {}
};

// ---------------------------------------------------------------------------
// Ghost fill
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fill_halo(GhostDev g, double* __restrict__ q, int plane) {
  const int row = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 4);
  const int lane = threadIdx.x & 15;
  if (row >= g.rows) return;   // whole 16-lane group leaves together
  const int b = g.ptr[row], e = g.ptr[row + 1];
  const double* q1 = q + plane;
  const double* q2 = q + 2 * (size_t)plane;
  double mass = 0, mu = 0, mv = 0;
  for (int k = b + lane; k < e; k += 16) {
    const int c = g.col[k];
    const double a0 = q[c], a1 = q1[c], a2 = q2[c];
    mass = fma(g.val[k], a0, mass);
    mu = fma(g.val[g.nnz + k], a1, fma(g.val[2 * g.nnz + k], a2, mu));
    mv = fma(g.val[3 * g.nnz + k], a1, fma(g.val[4 * g.nnz + k], a2, mv));
  }
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) {
    mass += __shfl_xor(mass, off, 16);
    mu += __shfl_xor(mu, off, 16);
    mv += __shfl_xor(mv, off, 16);
  }
  if (lane == 0) {
    const int d = g.dst[row];
    q[d] = mass;
    q[plane + d] = mu;
    q[2 * (size_t)plane + d] = mv;
  }
}

// ---------------------------------------------------------------------------
// Reconstruction of one cell.  Axis coordinates: 0 -> -1/2, 1 -> +1/2,
// 2+h -> Gauss node h.  Point numbering of one cell: x-edge left (h),
// x-edge right (h), y-edge bottom (h), y-edge top (h), CQP (v outer, h inner).
// ---------------------------------------------------------------------------
template <int K, bool W, int M>
struct Recon {
  static constexpr int R = (K - 1) / 2;
  static constexpr int L = (K + 1) / 2;     // sub-stencil width (WENO)
  static constexpr int S = L * L;
  static constexpr int NA = 2 + M;

  const double* __restrict__ c0;   // var-0 value of the cell
  int P;
  size_t vs;                       // distance between variables
  const CTab t;
  double kap[W ? 3 : 1][W ? S : 1];

  __device__ Recon(const double* c, int P_, size_t vs_, const CTab& t_) : c0(c), P(P_), vs(vs_), t(t_) {}

  __device__ __forceinline__ double at(int v, int dy, int dx) const { return c0[v * vs + dy * P + dx]; }

  // WENO: smoothness indicators, tau (3.24) and kappa_j = 1 + tau/(beta_j + eps) (3.23)
  __device__ void init() {
    if constexpr (W) {
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        double beta[S];
#pragma unroll
        for (int sx = 0; sx < L; ++sx) {
          double tr[2 * R + 1][L];
#pragma unroll
          for (int row = 0; row < 2 * R + 1; ++row)
#pragma unroll
            for (int al = 0; al < L; ++al) {
              double s = 0;
#pragma unroll
              for (int a = 0; a < L; ++a) s = fma(t.V[(sx * L + al) * L + a], at(v, row - R, sx - (L - 1) + a), s);
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
                for (int bb = 0; bb < L; ++bb) c = fma(t.V[(sy * L + be) * L + bb], tr[sy + bb][al], c);
                b = fma(t.lam[be * L + al] * c, c, b);
              }
            beta[sy * L + sx] = b;
          }
        }
        double tau = 0;
#pragma unroll
        for (int i = 0; i < S; ++i)
#pragma unroll
          for (int j = i + 1; j < S; ++j) tau += fabs(beta[i] - beta[j]);
        tau *= 2.0 / (S * (S + 1));
#pragma unroll
        for (int j = 0; j < S; ++j) kap[v][j] = 1.0 + tau / (beta[j] + t.eps);
      }
    }
  }

  // x-pass at axis px: TPP: xr[row] (2R+1 values); WENO: xr[sx][row] (L x (2R+1))
  __device__ __forceinline__ void xpass(int v, int px, double* xr) const {
    if constexpr (!W) {
#pragma unroll
      for (int row = 0; row < 2 * R + 1; ++row) {
        double s = 0;
#pragma unroll
        for (int a = 0; a < K; ++a) s = fma(t.wc[px * K + a], at(v, row - R, a - R), s);
        xr[row] = s;
      }
    } else {
#pragma unroll
      for (int sx = 0; sx < L; ++sx)
#pragma unroll
        for (int row = 0; row < 2 * R + 1; ++row) {
          double s = 0;
#pragma unroll
          for (int a = 0; a < L; ++a)
            s = fma(t.wsub[(sx * NA + px) * L + a], at(v, row - R, sx - (L - 1) + a), s);
          xr[sx * (2 * R + 1) + row] = s;
        }
    }
  }

  // value at (px, py) from the x-pass; pt = point number (for WENO weights)
  __device__ __forceinline__ double point(int v, int py, int pt, const double* xr) const {
    if constexpr (!W) {
      double s = 0;
#pragma unroll
      for (int b = 0; b < K; ++b) s = fma(t.wc[py * K + b], xr[b], s);
      return s;
    } else {
      double ap = 0, dp = 0, am = 0, dm = 0;
#pragma unroll
      for (int sy = 0; sy < L; ++sy)
#pragma unroll
        for (int sx = 0; sx < L; ++sx) {
          double p = 0;
#pragma unroll
          for (int b = 0; b < L; ++b) p = fma(t.wsub[(sy * NA + py) * L + b], xr[sx * (2 * R + 1) + sy + b], p);
          const int j = sy * L + sx;
          const double kp = kap[v][j];
          const double gpk = t.gp[pt * S + j] * kp, gmk = t.gm[pt * S + j] * kp;
          ap = fma(gpk, p, ap);
          dp += gpk;
          am = fma(gmk, p, am);
          dm += gmk;
        }
      // sigma+ sum w+ p - sigma- sum w- p, w = alpha / sum alpha
      return (t.sp[pt] * ap * dm - t.sm[pt] * am * dp) / (dp * dm);
    }
  }

  static constexpr int XR = W ? L * (2 * R + 1) : (2 * R + 1);

  // all m values of one side of the cell (0 left, 1 right, 2 bottom, 3 top), 3 vars
  __device__ void side(int sd, double out[3][M]) const {
    double xr[XR];
    if (sd < 2) {
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        xpass(v, sd, xr);
#pragma unroll
        for (int h = 0; h < M; ++h) out[v][h] = point(v, 2 + h, sd * M + h, xr);
      }
    } else {
#pragma unroll
      for (int h = 0; h < M; ++h)
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          xpass(v, 2 + h, xr);
          out[v][h] = point(v, sd - 2, (sd == 2 ? 2 * M : 3 * M) + h, xr);
        }
    }
  }
};

// ---------------------------------------------------------------------------
// LMARS flux (3.30)-(3.38) with upwind term |m|(q_R - q_L); dir 0 = x, 1 = y
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lmars(const double* qL, const double* qR, double X, double Y, int dir,
                                      double a, double* F) {
  const double X2 = X * X, Y2 = Y * Y;
  const double ox = 1.0 + X2, oy = 1.0 + Y2;
  const double d2 = ox + Y2;
  const double dl = sqrt(d2);
  const double idl = 1.0 / dl;
  const double sg = a * a * ox * oy * idl * idl * idl;             // (2.8)
  const double isg = 1.0 / sg;
  const double sgii = dl / (a * sqrt(dir == 0 ? ox : oy));         // sqrt(G^ii)
  const int iv = 1 + dir;
  const double phiL = qL[0] * isg, phiR = qR[0] * isg;
  const double upL = qL[iv] / (qL[0] * sgii);                      // (3.31)
  const double upR = qR[iv] / (qR[0] * sgii);
  const double c = 0.5 * (sqrt(phiL) + sqrt(phiR));                // (3.34)-(3.35)
  const double ms = 0.5 * (upL + upR - (phiR - phiL) / c);         // (3.32)
  const double ps = 0.5 * (phiL + phiR - c * (upR - upL));         // (3.33)
  const double mm = ms * sgii;                                     // (3.36)
  const double am = fabs(mm);
#pragma unroll
  for (int v = 0; v < 3; ++v) F[v] = 0.5 * (mm * (qL[v] + qR[v]) - am * (qR[v] - qL[v]));   // (3.37)
  const double pr = 0.5 * ps * ps * idl;                           // (3.38): sqrtG G^ij = (..)/delta
  if (dir == 0) {
    F[1] += pr * oy;
    F[2] += pr * X * Y;
  } else {
    F[1] += pr * X * Y;
    F[2] += pr * ox;
  }
}

// Metric (2.2) and Coriolis (2.3) sources at one point; L = c0 + cX X + cY Y
// so that f*delta = 2 Omega L.
__device__ __forceinline__ void sources(double Q0, double Q1, double Q2, double X, double Y, double Lc,
                                        double omega2, double& s1, double& s2) {
  const double X2 = X * X, Y2 = Y * Y;
  const double id2 = 1.0 / (1.0 + X2 + Y2);
  const double iq = 2.0 / Q0;
  const double m1 = iq * (-X * Y2 * Q1 * Q1 + Y * (1.0 + Y2) * Q1 * Q2);
  const double m2 = iq * (X * (1.0 + X2) * Q1 * Q2 - X2 * Y * Q2 * Q2);
  const double f = omega2 * Lc;
  const double c1 = f * (-X * Y * Q1 + (1.0 + Y2) * Q2);
  const double c2 = f * (-(1.0 + X2) * Q1 + X * Y * Q2);
  s1 = (m1 + c1) * id2;
  s2 = (m2 + c2) * id2;
}

// ---------------------------------------------------------------------------
// Panel-edge traces: bt[((A*4+side)*n + t)*m + h][var], in A's variables
// ---------------------------------------------------------------------------
template <int K, bool W, int M>
__global__ __launch_bounds__(64) void k_edge_traces(DevTables td, const double* __restrict__ q,
                                                     double* __restrict__ bt) {
  const CTab t(td);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 24 * t.n) return;
  const size_t vs = (size_t)6 * t.P * t.P;
  Recon<K, W, M> rc(q + t.bt_cell[idx], t.P, vs, t);
  rc.init();
  double vals[3][M];
  rc.side(t.bt_side[idx], vals);
  const int rev = t.bt_rev[idx];
#pragma unroll
  for (int h = 0; h < M; ++h) {
    const int hb = rev ? M - 1 - h : h;
    cdp cv = t.bt_conv + ((size_t)idx * M + h) * 5;
    double* o = bt + ((size_t)idx * M + h) * 3;
    o[0] = cv[0] * vals[0][hb];
    o[1] = cv[1] * vals[1][hb] + cv[2] * vals[2][hb];
    o[2] = cv[3] * vals[1][hb] + cv[4] * vals[2][hb];
  }
}

// ---------------------------------------------------------------------------
// Fused stage kernel
// ---------------------------------------------------------------------------
struct StageArgs {
  const double* q;
  const double* qn;
  double* out;
  const double* bt;
  double ca, cb, cc;
  int out_padded;
  int strip_w, seg_h, n_strips, n_segs;
};

// reciprocal: hardware estimate refined by two Newton-Raphson steps
__device__ __forceinline__ double rcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

// square root: Goldschmidt iteration from the hardware reciprocal square root
__device__ __forceinline__ double sqrt_g(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  return fma(d, h, g);
}

// LMARS with the fast reciprocal/root; X-direction (dir 0) or y (dir 1).
// sqx = sqrt(1 + X^2), sqy = sqrt(1 + Y^2) come from tables.
__device__ __forceinline__ void lmars_fast(const double* qL, const double* qR, double X, double Y, double sqx,
                                           double sqy, int dir, double a, double ia, double* F) {
  const double ox = sqx * sqx, oy = sqy * sqy;
  const double d2 = fma(X, X, oy);
  const double dl = sqrt_g(d2);
  const double idl = rcp(dl);
  // 1/sqrtG = delta^3 / (a^2 (1+X^2)(1+Y^2))
  const double isg = d2 * dl * ia * ia * rcp(ox * oy);
  const double sgii = dl * ia * rcp(dir == 0 ? sqx : sqy);      // sqrt(G^ii)
  const int iv = 1 + dir;
  const double phiL = qL[0] * isg, phiR = qR[0] * isg;
  const double iL = rcp(qL[0] * sgii), iR = rcp(qR[0] * sgii);
  const double upL = qL[iv] * iL, upR = qR[iv] * iR;              // (3.31)
  const double c = 0.5 * (sqrt_g(phiL) + sqrt_g(phiR));           // (3.34)-(3.35)
  const double ms = 0.5 * (upL + upR - (phiR - phiL) * rcp(c));   // (3.32)
  const double ps = 0.5 * (phiL + phiR - c * (upR - upL));        // (3.33)
  const double mm = ms * sgii;                                    // (3.36)
  const double am = fabs(mm);
#pragma unroll
  for (int v = 0; v < 3; ++v) F[v] = 0.5 * (mm * (qL[v] + qR[v]) - am * (qR[v] - qL[v]));   // (3.37)
  const double pr = 0.5 * ps * ps * idl;                          // (3.38)
  if (dir == 0) {
    F[1] = fma(pr, oy, F[1]);
    F[2] = fma(pr, X * Y, F[2]);
  } else {
    F[1] = fma(pr, X * Y, F[1]);
    F[2] = fma(pr, ox, F[2]);
  }
}

__device__ __forceinline__ void sources_fast(double Q0, double Q1, double Q2, double X, double Y, double Lc,
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

// Stencil window in LDS: NR = 2R+1 padded rows of CW = 64 + 2R columns of a
// strip, 3 variables; LDS column c holds padded column i0 - 1 + c.
template <int K, bool W, int M>
struct Window {
  static constexpr int R = (K - 1) / 2;
  static constexpr int L = (K + 1) / 2;
  static constexpr int S = L * L;
  static constexpr int NA = 2 + M;
  static constexpr int NR = 2 * R + 1;
  static constexpr int CW = 64 + 2 * R;
};

template <int K, bool W, int M>
#ifndef HOPE_STAGE_WAVES
#define HOPE_STAGE_WAVES 1
#endif
__global__ __launch_bounds__(64, HOPE_STAGE_WAVES) void k_stage(DevTables td, StageArgs A) {
  const CTab t(td);
  using Wd = Window<K, W, M>;
  constexpr int R = Wd::R, L = Wd::L, S = Wd::S, NA = Wd::NA, NR = Wd::NR, CW = Wd::CW;
  constexpr int XR = W ? L * NR : NR;
  __shared__ double sq[3][NR][CW];

  const int n = t.n, P = t.P;
  const size_t plane = (size_t)P * P;
  const size_t vs = 6 * plane;
  int item = blockIdx.x;
  const int seg = item % A.n_segs;
  item /= A.n_segs;
  const int strip = item % A.n_strips;
  const int p = item / A.n_strips;
  const int lane = threadIdx.x;
  const int i0 = strip * A.strip_w;
  const int i1 = min(n, i0 + A.strip_w);
  const int i = i0 - 1 + lane;
  const bool in_strip = (i >= i0 - 1) && (i <= i1);
  const bool real = in_strip && i >= 0 && i < n;
  const bool owner = i >= i0 && i < i1;
  const int j0 = seg * A.seg_h;
  const int j1 = min(n, j0 + A.seg_h);
  const double invd = t.inv_delta;
  const double ia = 1.0 / t.radius;
  const double* qp = A.q + p * plane;
  const double* btp = A.bt + (size_t)p * 4 * n * M * 3;
  const double Lx0 = t.fcoef[p * 3 + 0], LxX = t.fcoef[p * 3 + 1], LxY = t.fcoef[p * 3 + 2];
  const int ic = max(0, min(n - 1, i));        // clamped column for table reads
  const int ie = max(0, min(n, i));            // clamped edge index
  const double Xei = t.Xe[ie], sqxe = t.sqe[ie];

  // ---- window loading --------------------------------------------------
  constexpr int PER = (3 * CW + 63) / 64;
  auto fetch = [&](int pr, double* buf) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = lane + 64 * k;
      const int v = idx / CW, c = idx % CW;
      const int gc = i0 - 1 + c;
      buf[k] = (idx < 3 * CW && pr >= 0 && pr < P && gc >= 0 && gc < P) ? qp[v * vs + (size_t)pr * P + gc] : 0.0;
    }
  };
  auto store = [&](int pr, const double* buf) {
    const int slot = pr % NR;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = lane + 64 * k;
      if (idx < 3 * CW) sq[idx / CW][slot][idx % CW] = buf[k];
    }
  };
  // stencil value at offset (dy, dx) of this lane's cell in the row centred at padded row pc
  // pc = interior row of the centre cell, so the padded row is pc + R + dy
  auto at = [&](int v, int pc, int dy, int dx) -> double { return sq[v][(pc + R + dy) % NR][lane + R + dx]; };

  // ---- reconstruction helpers (centre padded row pc) --------------------
  double kap[W ? 3 : 1][W ? S : 1];
  auto weights_init = [&](int pc) {
    if constexpr (W) {
#pragma unroll
      for (int v = 0; v < 3; ++v) {
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
              for (int a = 0; a < L; ++a)
                s = fma(t.V[(sx * L + al) * L + a], at(v, pc, row - R, sx - (L - 1) + a), s);
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
                for (int bb = 0; bb < L; ++bb) c = fma(t.V[(sy * L + be) * L + bb], tr[sy + bb][al], c);
                b = fma(t.lam[be * L + al] * c, c, b);
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
        for (int j = 0; j < S; ++j) kap[v][j] = fma(tau, rcp(beta[j] + t.eps), 1.0);
      }
    }
  };
  auto xpass = [&](int v, int pc, int px, double* xr) {
    // each pass re-reads its stencil from LDS rather than keeping all of it live
    asm volatile("" ::: "memory");
    if constexpr (!W) {
#pragma unroll
      for (int row = 0; row < NR; ++row) {
        double s = 0;
#pragma unroll
        for (int a = 0; a < K; ++a) s = fma(t.wc[px * K + a], at(v, pc, row - R, a - R), s);
        xr[row] = s;
      }
    } else {
#pragma unroll
      for (int sx = 0; sx < L; ++sx)
#pragma unroll
        for (int row = 0; row < NR; ++row) {
          double s = 0;
#pragma unroll
          for (int a = 0; a < L; ++a)
            s = fma(t.wsub[(sx * NA + px) * L + a], at(v, pc, row - R, sx - (L - 1) + a), s);
          xr[sx * NR + row] = s;
        }
    }
  };
  auto point = [&](int v, int py, int pt, const double* xr) -> double {
    if constexpr (!W) {
      double s = 0;
#pragma unroll
      for (int b = 0; b < K; ++b) s = fma(t.wc[py * K + b], xr[b], s);
      return s;
    } else {
      double ap = 0, dp = 0, am = 0, dm = 0;
#pragma unroll
      for (int sy = 0; sy < L; ++sy)
#pragma unroll
        for (int sx = 0; sx < L; ++sx) {
          double pv = 0;
#pragma unroll
          for (int b = 0; b < L; ++b) pv = fma(t.wsub[(sy * NA + py) * L + b], xr[sx * NR + sy + b], pv);
          const int j = sy * L + sx;
          const double tk = kap[v][j] * pv;
          ap = fma(t.gp[pt * S + j], tk, ap);
          am = fma(t.gm[pt * S + j], tk, am);
          dp = fma(t.gp[pt * S + j], kap[v][j], dp);
          dm = fma(t.gm[pt * S + j], kap[v][j], dm);
        }
      return (t.sp[pt] * ap * dm - t.sm[pt] * am * dp) * rcp(dp * dm);
    }
  };

  // ---- prologue: window and the top traces of row j0-1 ------------------
  double ptop[3][M];
  double nxt[PER];
  {
    for (int pr = max(0, j0 - 1); pr < j0 + 2 * R; ++pr) {
      fetch(pr, nxt);
      store(pr, nxt);
    }
    fetch(j0 + 2 * R, nxt);          // row needed by the first step
  }
  __syncthreads();
  if (j0 == 0) {
#pragma unroll
    for (int h = 0; h < M; ++h)
#pragma unroll
      for (int v = 0; v < 3; ++v) ptop[v][h] = real ? btp[(((size_t)2 * n + ic) * M + h) * 3 + v] : 1.0;
  } else {
    weights_init(j0 - 1);
#pragma unroll
    for (int h = 0; h < M; ++h)
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        double xr[XR];
        xpass(v, j0 - 1, 2 + h, xr);
        ptop[v][h] = point(v, 1, 3 * M + h, xr);
      }
  }
  double acc[3] = {0.0, 0.0, 0.0};

  for (int j = j0; j <= j1; ++j) {
    const bool last = (j == j1);
    const int pc = j;
    // the window of step j holds padded rows j .. j+2R; row j+2R was fetched
    // during the previous step and replaces row j-1, no longer read
    const bool have = !(last && j1 == n) && (j + 2 * R) < P;
    __syncthreads();
    if (have) store(j + 2 * R, nxt);
    __syncthreads();
    const bool want = (j + 1 < j1 || (j + 1 == j1 && j1 < n)) && (j + 2 * R + 1) < P;
    if (want) fetch(j + 2 * R + 1, nxt);
    double gb[3] = {0.0, 0.0, 0.0};
    double fl[3] = {0.0, 0.0, 0.0};
    double s1 = 0.0, s2 = 0.0;
    if (!last) {
      weights_init(pc);
      // x-edges: left trace (px = 0), right trace (px = 1), flux through the left edge
      double xl[3][M], xrt[3][M];
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        double xr[XR];
        xpass(v, pc, 0, xr);
#pragma unroll
        for (int h = 0; h < M; ++h) xl[v][h] = point(v, 2 + h, h, xr);
        xpass(v, pc, 1, xr);
#pragma unroll
        for (int h = 0; h < M; ++h) xrt[v][h] = point(v, 2 + h, M + h, xr);
      }
#pragma unroll
      for (int h = 0; h < M; ++h) {
        double qL[3], qR[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          qL[v] = __shfl_up(xrt[v][h], 1, 64);
          qR[v] = xl[v][h];
        }
        if (i == 0) {
#pragma unroll
          for (int v = 0; v < 3; ++v) qL[v] = btp[(((size_t)0 * n + j) * M + h) * 3 + v];
        }
        if (i == n) {
#pragma unroll
          for (int v = 0; v < 3; ++v) qR[v] = btp[(((size_t)1 * n + j) * M + h) * 3 + v];
        }
        if (!(in_strip && i >= 0 && i <= n && lane >= 1)) {
#pragma unroll
          for (int v = 0; v < 3; ++v) qL[v] = qR[v] = (v == 0) ? 1.0 : 0.0;
        }
        double F[3];
        const double Y = t.Xg[j * M + h];
        lmars_fast(qL, qR, Xei, Y, sqxe, t.sqg[j * M + h], 0, t.radius, ia, F);
#pragma unroll
        for (int v = 0; v < 3; ++v) fl[v] = fma(t.gw[h], F[v], fl[v]);
      }
      // Gauss-node columns: y-edge traces, y-flux through the bottom edge, CQP sources
#pragma unroll
      for (int h = 0; h < M; ++h) {
        double yb[3], yt[3], cq[3][M];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          double xr[XR];
          xpass(v, pc, 2 + h, xr);
          yb[v] = point(v, 0, 2 * M + h, xr);
          yt[v] = point(v, 1, 3 * M + h, xr);
#pragma unroll
          for (int w = 0; w < M; ++w) cq[v][w] = point(v, 2 + w, 4 * M + w * M + h, xr);
        }
        const double X = t.Xg[ic * M + h];
        const double sqx = t.sqg[ic * M + h];
        if (!real) {
          yb[0] = ptop[0][h] = 1.0;
          yb[1] = yb[2] = ptop[1][h] = ptop[2][h] = 0.0;
#pragma unroll
          for (int w = 0; w < M; ++w) { cq[0][w] = 1.0; cq[1][w] = cq[2][w] = 0.0; }
        }
        double qL[3] = {ptop[0][h], ptop[1][h], ptop[2][h]};
        double F[3];
        lmars_fast(qL, yb, X, t.Xe[j], sqx, t.sqe[j], 1, t.radius, ia, F);
#pragma unroll
        for (int v = 0; v < 3; ++v) gb[v] = fma(t.gw[h], F[v], gb[v]);
#pragma unroll
        for (int v = 0; v < 3; ++v) ptop[v][h] = yt[v];
#pragma unroll
        for (int w = 0; w < M; ++w) {
          const double Y = t.Xg[j * M + w];
          double a1, a2;
          sources_fast(cq[0][w], cq[1][w], cq[2][w], X, Y, Lx0 + LxX * X + LxY * Y, t.omega2, a1, a2);
          const double gw = t.gw[h] * t.gw[w];
          s1 = fma(gw, a1, s1);
          s2 = fma(gw, a2, s2);
        }
      }
    } else {
      // epilogue: bottom traces of row j1 and the flux through the top edge of row j1-1
      double yb[3][M];
      if (j1 == n) {
#pragma unroll
        for (int h = 0; h < M; ++h)
#pragma unroll
          for (int v = 0; v < 3; ++v) yb[v][h] = real ? btp[(((size_t)3 * n + ic) * M + h) * 3 + v] : (v ? 0.0 : 1.0);
      } else {
        weights_init(pc);
#pragma unroll
        for (int h = 0; h < M; ++h)
#pragma unroll
          for (int v = 0; v < 3; ++v) {
            double xr[XR];
            xpass(v, pc, 2 + h, xr);
            yb[v][h] = point(v, 0, 2 * M + h, xr);
          }
      }
#pragma unroll
      for (int h = 0; h < M; ++h) {
        double qL[3] = {ptop[0][h], ptop[1][h], ptop[2][h]};
        double qR[3] = {yb[0][h], yb[1][h], yb[2][h]};
        if (!real) {
          qL[0] = qR[0] = 1.0;
          qL[1] = qL[2] = qR[1] = qR[2] = 0.0;
        }
        double F[3];
        lmars_fast(qL, qR, t.Xg[ic * M + h], t.Xe[j], t.sqg[ic * M + h], t.sqe[j], 1, t.radius, ia, F);
#pragma unroll
        for (int v = 0; v < 3; ++v) gb[v] = fma(t.gw[h], F[v], gb[v]);
      }
    }
    // ---- finalize row j-1 ---------------------------------------------------
    if (j > j0 && owner) {
      const int jr = j - 1;
      const size_t c_in = (size_t)(jr + R) * P + (i + R);
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        const double dq = fma(-gb[v], invd, acc[v]);
        const size_t o_in = v * vs + p * plane + c_in;
        double val = A.cc * dq;
        if (A.cb != 0.0) val = fma(A.cb, A.q[o_in], val);
        if (A.qn) val = fma(A.ca, A.qn[o_in], val);
        if (A.out_padded) {
          A.out[o_in] = val;
        } else {
          A.out[((size_t)(v * 6 + p) * n + jr) * n + i] = val;
        }
      }
    }
    if (last) break;
    double fr[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) fr[v] = __shfl_down(fl[v], 1, 64);
    acc[0] = (fl[0] - fr[0] + gb[0]) * invd;
    acc[1] = fma(fl[1] - fr[1] + gb[1], invd, s1);
    acc[2] = fma(fl[2] - fr[2] + gb[2], invd, s2);
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
int launch_fill_halo(const GhostDev& g, double* q, int plane, void* stream) {
  if (g.rows == 0) return 0;
  const int threads = 256;
  const int blocks = (int)(((size_t)g.rows * 16 + threads - 1) / threads);
  hipLaunchKernelGGL(k_fill_halo, dim3(blocks), dim3(threads), 0, (hipStream_t)stream, g, q, plane);
  return (int)hipGetLastError();
}

template <int K, bool W, int M>
static int edge_traces_t(const DevTables& t, const double* q, double* bt, void* stream) {
  const int total = 24 * t.n;
  hipLaunchKernelGGL((k_edge_traces<K, W, M>), dim3((total + 63) / 64), dim3(64), 0, (hipStream_t)stream, t, q,
                     bt);
  return (int)hipGetLastError();
}

template <int K, bool W, int M>
static int stage_t(const DevTables& t, const StageArgs& a, void* stream) {
  const int items = 6 * a.n_strips * a.n_segs;
  hipLaunchKernelGGL((k_stage<K, W, M>), dim3(items), dim3(64), 0, (hipStream_t)stream, t, a);
  return (int)hipGetLastError();
}

#define HOPE_DISPATCH(FN, ...)                                    \
  do {                                                            \
    if (!weno) {                                                  \
      switch (k) {                                                \
        case 3: return FN<3, false, 2>(__VA_ARGS__);              \
        case 5: return FN<5, false, 3>(__VA_ARGS__);              \
        case 7: return FN<7, false, 4>(__VA_ARGS__);              \
        case 9: return FN<9, false, 5>(__VA_ARGS__);              \
        case 11: return FN<11, false, 6>(__VA_ARGS__);            \
        case 13: return FN<13, false, 7>(__VA_ARGS__);            \
      }                                                           \
    } else {                                                      \
      switch (k) {                                                \
        case 3: return FN<3, true, 2>(__VA_ARGS__);               \
        case 5: return FN<5, true, 3>(__VA_ARGS__);               \
      }                                                           \
    }                                                             \
    return (int)hipErrorInvalidValue;                             \
  } while (0)

int launch_edge_traces(int k, int weno, const DevTables& t, const double* q, double* bt, void* stream) {
  HOPE_DISPATCH(edge_traces_t, t, q, bt, stream);
}

int launch_stage(int k, int weno, const DevTables& t, const double* q, const double* qn, double* out,
                 int out_padded, double ca, double cb, double cc, const double* bt, int strip_w, int seg_h,
                 void* stream) {
  StageArgs a;
  a.q = q;
  a.qn = qn;
  a.out = out;
  a.bt = bt;
  a.ca = ca;
  a.cb = cb;
  a.cc = cc;
  a.out_padded = out_padded;
  a.strip_w = strip_w;
  a.seg_h = seg_h;
  a.n_strips = (t.n + strip_w - 1) / strip_w;
  a.n_segs = (t.n + seg_h - 1) / seg_h;
  HOPE_DISPATCH(stage_t, t, a, stream);
}

}  // namespace hope
