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
  const DevTables t;
  double kap[W ? 3 : 1][W ? S : 1];

  __device__ Recon(const double* c, int P_, size_t vs_, const DevTables& t_) : c0(c), P(P_), vs(vs_), t(t_) {}

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
__global__ __launch_bounds__(64) void k_edge_traces(DevTables t, const double* __restrict__ q,
                                                     double* __restrict__ bt) {
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
    const double* cv = t.bt_conv + ((size_t)idx * M + h) * 5;
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

template <int K, bool W, int M>
__global__ __launch_bounds__(64) void k_stage(DevTables t, StageArgs A) {
  using RC = Recon<K, W, M>;
  const int n = t.n, P = t.P, r = t.r;
  const size_t plane = (size_t)P * P;
  const size_t vs = 6 * plane;
  int item = blockIdx.x;
  const int seg = item % A.n_segs;
  item /= A.n_segs;
  const int strip = item % A.n_strips;
  const int p = item / A.n_strips;
  const int lane = threadIdx.x;
  const int i0 = strip * A.strip_w;
  const int i1 = min(n, i0 + A.strip_w);          // owned columns [i0, i1)
  const int i = i0 - 1 + lane;                     // this lane's column
  const bool in_strip = (i >= i0 - 1) && (i <= i1);
  const bool can_rec = in_strip && i >= 0 && i < n;      // a real cell of this panel
  const bool owner = i >= i0 && i < i1;
  const int j0 = seg * A.seg_h;
  const int j1 = min(n, j0 + A.seg_h);
  const double invd = t.inv_delta;
  const double* qp = A.q + p * plane;
  const double* btp = A.bt + (size_t)p * 4 * n * M * 3;
  const double Lx0 = t.fcoef[p * 3 + 0], LxX = t.fcoef[p * 3 + 1], LxY = t.fcoef[p * 3 + 2];

  // ---- prologue: top traces of row j0-1 --------------------------------
  double ptop[3][M];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int h = 0; h < M; ++h) ptop[v][h] = 0.0;
  if (i >= 0 && i < n && in_strip) {
    if (j0 == 0) {
#pragma unroll
      for (int h = 0; h < M; ++h)
#pragma unroll
        for (int v = 0; v < 3; ++v) ptop[v][h] = btp[(((size_t)2 * n + i) * M + h) * 3 + v];
    } else {
      RC rc(qp + (size_t)(j0 - 1 + r) * P + (i + r), P, vs, t);
      rc.init();
      rc.side(3, ptop);
    }
  }
  double acc[3] = {0.0, 0.0, 0.0};

  for (int j = j0; j <= j1; ++j) {
    const bool last = (j == j1);
    double xl[3][M], xrr[3][M], yb[3][M], yt[3][M];
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
      for (int h = 0; h < M; ++h) xl[v][h] = xrr[v][h] = yb[v][h] = yt[v][h] = 0.0;
    if (!last) {
      if (can_rec) {
        RC rc(qp + (size_t)(j + r) * P + (i + r), P, vs, t);
        rc.init();
        double xr[RC::XR];
        // x-edges
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          rc.xpass(v, 0, xr);
#pragma unroll
          for (int h = 0; h < M; ++h) xl[v][h] = rc.point(v, 2 + h, h, xr);
          rc.xpass(v, 1, xr);
#pragma unroll
          for (int h = 0; h < M; ++h) xrr[v][h] = rc.point(v, 2 + h, M + h, xr);
        }
        // Gauss-node columns: y-edges and CQPs
#pragma unroll
        for (int h = 0; h < M; ++h) {
          double cq[3][M];
#pragma unroll
          for (int v = 0; v < 3; ++v) {
            rc.xpass(v, 2 + h, xr);
            yb[v][h] = rc.point(v, 0, 2 * M + h, xr);
            yt[v][h] = rc.point(v, 1, 3 * M + h, xr);
#pragma unroll
            for (int w = 0; w < M; ++w) cq[v][w] = rc.point(v, 2 + w, 4 * M + w * M + h, xr);
          }
          const double X = t.Xg[i * M + h];
#pragma unroll
          for (int w = 0; w < M; ++w) {
            const double Y = t.Xg[j * M + w];
            double a1, a2;
            sources(cq[0][w], cq[1][w], cq[2][w], X, Y, Lx0 + LxX * X + LxY * Y, t.omega2, a1, a2);
            const double gw = t.gw[h] * t.gw[w];
            s1 = fma(gw, a1, s1);
            s2 = fma(gw, a2, s2);
          }
        }
      }
    } else {
      // epilogue: bottom traces of row j1 (the row above the segment)
      if (i >= 0 && i < n && in_strip) {
        if (j1 == n) {
#pragma unroll
          for (int h = 0; h < M; ++h)
#pragma unroll
            for (int v = 0; v < 3; ++v) yb[v][h] = btp[(((size_t)3 * n + i) * M + h) * 3 + v];
        } else {
          RC rc(qp + (size_t)(j1 + r) * P + (i + r), P, vs, t);
          rc.init();
          rc.side(2, yb);
        }
      }
    }
    // ---- y-flux through the bottom edge of (i, j) ------------------------
    double gb[3] = {0.0, 0.0, 0.0};
    if (i >= 0 && i < n && in_strip) {
      const double Ye = t.Xe[j];
#pragma unroll
      for (int h = 0; h < M; ++h) {
        double qL[3] = {ptop[0][h], ptop[1][h], ptop[2][h]};
        double qR[3] = {yb[0][h], yb[1][h], yb[2][h]};
        double F[3];
        lmars(qL, qR, t.Xg[i * M + h], Ye, 1, t.radius, F);
#pragma unroll
        for (int v = 0; v < 3; ++v) gb[v] = fma(t.gw[h], F[v], gb[v]);
      }
    }
    // ---- finalize row j-1 -------------------------------------------------
    if (j > j0 && owner) {
      const int jr = j - 1;
      const size_t c_in = (size_t)(jr + r) * P + (i + r);
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        const double dq = acc[v] - gb[v] * invd;
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
    // ---- x-flux through the left edge of each lane ------------------------
    double fl[3] = {0.0, 0.0, 0.0};
    {
      const double Xe = t.Xe[max(0, min(n, i))];
#pragma unroll
      for (int h = 0; h < M; ++h) {
        double qL[3], qR[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          qL[v] = __shfl_up(xrr[v][h], 1, 64);
          qR[v] = xl[v][h];
        }
        if (i == 0) {
#pragma unroll
          for (int v = 0; v < 3; ++v) qL[v] = btp[(((size_t)0 * n + j) * M + h) * 3 + v];
        }
        if (i == n && in_strip) {
#pragma unroll
          for (int v = 0; v < 3; ++v) qR[v] = btp[(((size_t)1 * n + j) * M + h) * 3 + v];
        }
        if (in_strip && i >= 0 && i <= n && lane >= 1) {
          double F[3];
          lmars(qL, qR, Xe, t.Xg[j * M + h], 0, t.radius, F);
#pragma unroll
          for (int v = 0; v < 3; ++v) fl[v] = fma(t.gw[h], F[v], fl[v]);
        }
      }
    }
    double fr[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) fr[v] = __shfl_down(fl[v], 1, 64);
    // ---- partial tendency of row j ------------------------------------------
    acc[0] = -(fr[0] - fl[0]) * invd + gb[0] * invd;
    acc[1] = -(fr[1] - fl[1]) * invd + gb[1] * invd + s1;
    acc[2] = -(fr[2] - fl[2]) * invd + gb[2] * invd + s2;
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
      for (int h = 0; h < M; ++h) ptop[v][h] = yt[v][h];
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
