// Device bodies of the HOPE right-hand-side kernels, shared by the kernels of
// one grid (kernels.hip) and the batched ensemble kernels (batch.hip).
//
//  halo_row    one row of the ghost fill g = G q (appendix (7.12))
//  edge_trace  at one panel-edge side, the neighbour panel's own trace,
//              converted into this panel's variables (3.26)-(3.29)
//  stage_tile  one work item of the fused stage: reconstruction (TPP (3.14)
//              or genuine 2D WENO (3.16)-(3.25)), LMARS (3.30)-(3.38), Gauss
//              quadrature (3.5)-(3.6) with sources (2.2)-(2.3), the tendency
//              (3.1) and an optional Runge-Kutta combination
//
// stage_tile marches: one wavefront owns a strip of up to 62 interior columns
// of one panel (lanes 1..62; lanes 0 and 63 are the strip's ring columns) and
// a segment of rows, walking up the rows.  The 2r+1 stencil rows of the strip
// sit in an LDS ring buffer (one new row per step, fetched a step ahead).  At
// each row every lane reconstructs its cell; the flux through the left edge
// of lane L takes the left state from lane L-1 by a cross-lane shuffle, and
// the flux through the bottom edge takes the top trace of the row below, kept
// from the previous step.  No trace goes to HBM.
//
// The grid's constant tables are one buffer read through the constant address
// space: with uniform addresses those reads are scalar loads into SGPRs.
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace hope {

// one ghost row of g = G q, reduced over 16 lanes (lane = 0..15 of the group)
__device__ __forceinline__ void halo_row(const GhostDev& g, double* __restrict__ q, size_t plane, int row, int lane) {
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

// the converted neighbour trace at the panel-edge side idx (0 <= idx < 24 n)
template <int K, bool W, int M>
__device__ __forceinline__ void edge_trace(cdp tab, cip itab, const GridScalars& gs, const double* __restrict__ q,
                                           double* __restrict__ bt, int idx) {
  using C = Cfg<K, W, M>;
  const int n = gs.n, P = gs.P;
  const TabOffsets O = tab_offsets(K, W, M, n);
  const size_t vs = (size_t)6 * P * P;
  const double* c0 = q + itab[O.i_cell + idx];
  const int sd = itab[O.i_side + idx];
  const int rev = itab[O.i_rev + idx];
  double vals[3][M];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    auto at = [&](int dy, int dx) -> double { return c0[v * vs + dy * P + dx]; };
    double kap[W ? C::S : 1];
    if constexpr (W) weno_kappa<K, W, M>(tab, gs.eps, at, [&](int j, double x) { kap[j] = x; });
    auto kf = [&](int j) -> double { return kap[j]; };
    double xr[C::XR];
    if (sd < 2) {
      xpass<K, W, M>(tab, sd, at, xr);
#pragma unroll
      for (int h = 0; h < M; ++h) vals[v][h] = point<K, W, M>(tab, 2 + h, sd * M + h, xr, kf);
    } else {
#pragma unroll
      for (int h = 0; h < M; ++h) {
        xpass<K, W, M>(tab, 2 + h, at, xr);
        vals[v][h] = point<K, W, M>(tab, sd - 2, (sd == 2 ? 2 * M : 3 * M) + h, xr, kf);
      }
    }
  }
#pragma unroll
  for (int h = 0; h < M; ++h) {
    const int hb = rev ? M - 1 - h : h;
    cdp cv = tab + O.bt_conv + ((size_t)idx * M + h) * 5;
    double* o = bt + ((size_t)idx * M + h) * 3;
    o[0] = cv[0] * vals[0][hb];
    o[1] = cv[1] * vals[1][hb] + cv[2] * vals[2][hb];
    o[2] = cv[3] * vals[1][hb] + cv[4] * vals[2][hb];
  }
}

struct StageArgs {
  const double* q;
  const double* qn;
  double* out;
  const double* bt;
  double ca, cb, cc;
  int out_padded;
  int strip_w, seg_h, n_strips, n_segs;
};

#ifndef HOPE_STAGE_WAVES
#define HOPE_STAGE_WAVES 1
#endif

template <int K, bool W, int M>
struct StageSmem {
  static constexpr int R = (K - 1) / 2, NR = 2 * R + 1, CW = 64 + 2 * R, S = ((K + 1) / 2) * ((K + 1) / 2);
  // stencil window: NR padded rows of CW columns (LDS column c = padded column i0-1+c)
  double sq[3][NR][CW];
  // WENO weights kappa_j per variable and lane, and the carried top traces
  double skap[W ? 3 : 1][W ? S : 1][64];
  double sptop[3][M][64];
};

// one work item (panel, strip, segment) of the fused stage; fcb = the 6 x 3
// Coriolis coefficients of the grid (or of one ensemble member)
template <int K, bool W, int M>
__device__ __forceinline__ void stage_tile(const double* __restrict__ tab_, cdp fcb, const GridScalars& gs,
                                           const StageArgs& A, int item, StageSmem<K, W, M>& sm) {
  using C = Cfg<K, W, M>;
  constexpr int R = C::R, S = C::S, NR = C::NR, XR = C::XR;
  constexpr int CW = 64 + 2 * R;
  auto& sq = sm.sq;
  auto& skap = sm.skap;
  auto& sptop = sm.sptop;
  const cdp tab = (cdp)tab_;
  const cdp ltab = tab;
  const int n = gs.n, P = gs.P;
  const TabOffsets O = tab_offsets(K, W, M, n);
  const size_t plane = (size_t)P * P;
  const size_t vs = 6 * plane;
  const int seg = item % A.n_segs;
  item /= A.n_segs;
  const int strip = item % A.n_strips;
  const int p = item / A.n_strips;
  const int lane = threadIdx.x;
  const int i0 = strip * A.strip_w;
  const int i1 = min(n, i0 + A.strip_w);          // owned columns [i0, i1)
  const int i = i0 - 1 + lane;                     // this lane's column
  const bool in_strip = (i >= i0 - 1) && (i <= i1);
  const bool real = in_strip && i >= 0 && i < n;   // a cell this lane can reconstruct
  const bool owner = i >= i0 && i < i1;            // a cell whose result this lane writes
  const int j0 = seg * A.seg_h;
  const int j1 = min(n, j0 + A.seg_h);
  const double invd = gs.inv_delta;
  const double ia = 1.0 / gs.radius;
  const double* qp = A.q + p * plane;
  const double* btp = A.bt + (size_t)p * 4 * n * M * 3;
  cdp fc = fcb + p * 3;
  const double Lx0 = fc[0], LxX = fc[1], LxY = fc[2];
  const int ic = max(0, min(n - 1, i));            // clamped column for table reads
  const int ie = max(0, min(n, i));                // clamped edge index
  const double Xei = tab[O.Xe + ie], sqxe = tab[O.sqe + ie];
  const bool xdead = !(in_strip && i >= 0 && i <= n && lane >= 1);   // no x-edge flux on this lane
  cdp Xg = tab + O.Xg, sqg = tab + O.sqg, Xe = tab + O.Xe, sqe = tab + O.sqe, gw = tab + C::O.gw;

  // ---- window rows ---------------------------------------------------------
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
  // stencil of variable v at offset (dy, dx) of this lane's cell in interior row pc
  auto win = [&](int v, int pc) {
    return [&, v, pc](int dy, int dx) -> double { return sq[v][(pc + R + dy) % NR][lane + R + dx]; };
  };
  auto kapv = [&](int v) {
    return [&, v](int j) -> double { return skap[v][j][lane]; };
  };
  auto weights = [&](int pc) {
    if constexpr (W) {
#pragma unroll 1
      for (int v = 0; v < 3; ++v) {
        asm volatile("" ::: "memory");
        weno_kappa<K, W, M>(ltab, gs.eps, win(v, pc), [&](int j, double x) { skap[v][j][lane] = x; });
      }
    }
  };
  // each pass re-reads its stencil from LDS rather than keeping all of it live
  auto pass = [&](int v, int pc, int px, double* xr) {
    asm volatile("" ::: "memory");
    xpass<K, W, M>(ltab, px, win(v, pc), xr);
  };
  auto ptop = [&](int v, int h) -> double& { return sptop[v][h][lane]; };

  // ---- prologue: window and the top traces of row j0-1 ------------------
  double nxt[PER];
  for (int pr = max(0, j0 - 1); pr < j0 + 2 * R; ++pr) {
    fetch(pr, nxt);
    store(pr, nxt);
  }
  fetch(j0 + 2 * R, nxt);          // row needed by the first step
  __syncthreads();
  if (j0 == 0) {
#pragma unroll
    for (int h = 0; h < M; ++h)
#pragma unroll
      for (int v = 0; v < 3; ++v) ptop(v, h) = real ? btp[(((size_t)2 * n + ic) * M + h) * 3 + v] : (v ? 0.0 : 1.0);
  } else {
    weights(j0 - 1);
#pragma unroll 1
    for (int h = 0; h < M; ++h)
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        double xr[XR];
        pass(v, j0 - 1, 2 + h, xr);
        ptop(v, h) = point<K, W, M>(ltab, 1, 3 * M + h, xr, kapv(v));
      }
  }
  double acc[3] = {0.0, 0.0, 0.0};

  for (int j = j0; j <= j1; ++j) {
    const bool last = (j == j1);
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
      weights(j);
      // x-edges: left trace (px = 0), right trace (px = 1), flux through the left edge
      double xl[3][M], xrt[3][M];
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        double xr[XR];
        pass(v, j, 0, xr);
#pragma unroll
        for (int h = 0; h < M; ++h) xl[v][h] = point<K, W, M>(ltab, 2 + h, h, xr, kapv(v));
        pass(v, j, 1, xr);
#pragma unroll
        for (int h = 0; h < M; ++h) xrt[v][h] = point<K, W, M>(ltab, 2 + h, M + h, xr, kapv(v));
      }
#pragma unroll
      for (int h = 0; h < M; ++h) {
        double qL[3], qR[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          qL[v] = __shfl_up(xrt[v][h], 1, 64);
          qR[v] = xl[v][h];
        }
        // panel edges take the neighbour's converted trace; lanes without an
        // edge of their own get a harmless state (selects, not branches: a
        // branch here splits the region and the register allocation suffers)
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          const double bl = btp[(((size_t)0 * n + j) * M + h) * 3 + v];
          const double br = btp[(((size_t)1 * n + j) * M + h) * 3 + v];
          const double dflt = v == 0 ? 1.0 : 0.0;
          qL[v] = xdead ? dflt : (i == 0 ? bl : qL[v]);
          qR[v] = xdead ? dflt : (i == n ? br : qR[v]);
        }
        double F[3];
        lmars(qL, qR, Xei, Xg[j * M + h], sqxe, sqg[j * M + h], 0, ia, F);
#pragma unroll
        for (int v = 0; v < 3; ++v) fl[v] = fma(gw[h], F[v], fl[v]);
      }
      // Gauss-node columns: y-edge traces, y-flux through the bottom edge, CQP sources
#pragma unroll 1
      for (int h = 0; h < M; ++h) {
        double yb[3], yt[3], cq[3][M];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          double xr[XR];
          pass(v, j, 2 + h, xr);
          yb[v] = point<K, W, M>(ltab, 0, 2 * M + h, xr, kapv(v));
          yt[v] = point<K, W, M>(ltab, 1, 3 * M + h, xr, kapv(v));
#pragma unroll
          for (int w = 0; w < M; ++w) cq[v][w] = point<K, W, M>(ltab, 2 + w, 4 * M + w * M + h, xr, kapv(v));
        }
        const double X = Xg[ic * M + h];
        const double sqx = sqg[ic * M + h];
        double qL[3] = {ptop(0, h), ptop(1, h), ptop(2, h)};
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          const double dflt = v == 0 ? 1.0 : 0.0;
          qL[v] = real ? qL[v] : dflt;
          yb[v] = real ? yb[v] : dflt;
#pragma unroll
          for (int w = 0; w < M; ++w) cq[v][w] = real ? cq[v][w] : dflt;
        }
        double F[3];
        lmars(qL, yb, X, Xe[j], sqx, sqe[j], 1, ia, F);
#pragma unroll
        for (int v = 0; v < 3; ++v) gb[v] = fma(gw[h], F[v], gb[v]);
#pragma unroll
        for (int v = 0; v < 3; ++v) ptop(v, h) = yt[v];
#pragma unroll
        for (int w = 0; w < M; ++w) {
          const double Y = Xg[j * M + w];
          double a1, a2;
          sources(cq[0][w], cq[1][w], cq[2][w], X, Y, Lx0 + LxX * X + LxY * Y, gs.omega2, a1, a2);
          const double g2 = gw[h] * gw[w];
          s1 = fma(g2, a1, s1);
          s2 = fma(g2, a2, s2);
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
        weights(j);
#pragma unroll
        for (int h = 0; h < M; ++h)
#pragma unroll
          for (int v = 0; v < 3; ++v) {
            double xr[XR];
            pass(v, j, 2 + h, xr);
            yb[v][h] = point<K, W, M>(ltab, 0, 2 * M + h, xr, kapv(v));
          }
      }
#pragma unroll
      for (int h = 0; h < M; ++h) {
        double qL[3], qR[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          const double dflt = v == 0 ? 1.0 : 0.0;
          qL[v] = real ? ptop(v, h) : dflt;
          qR[v] = real ? yb[v][h] : dflt;
        }
        double F[3];
        lmars(qL, qR, Xg[ic * M + h], Xe[j], sqg[ic * M + h], sqe[j], 1, ia, F);
#pragma unroll
        for (int v = 0; v < 3; ++v) gb[v] = fma(gw[h], F[v], gb[v]);
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

}  // namespace hope
