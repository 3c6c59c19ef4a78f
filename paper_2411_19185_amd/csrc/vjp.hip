// Adjoint (vector-Jacobian product) of the HOPE tendency, hand-written.
//
// Given w = dL/d(dq/dt) the kernels compute dL/dq in reverse order of the
// forward evaluation:
//   k_vjp_traces    recompute every cell's values at its edge and cell Gauss
//                   points (the forward reconstruction) into scratch T
//   k_vjp_points    the cotangent of every point value: per cell edge, the
//                   adjoint of the LMARS flux (3.30)-(3.38) at its Gauss
//                   points (flux cotangent from the tendency (3.1) and the
//                   quadrature (3.5)) for the traces on both sides; per cell,
//                   that of the sources (2.2)-(2.3) at its nodes (3.6)
//   k_vjp_edges     adds, at every panel-edge point, the adjoint of the
//                   neighbour panel's own flux with respect to the converted
//                   trace, taken back through the transposed conversion
//                   (3.26)-(3.29)
//   k_vjp_weno      WENO: cotangents of the stencil cell values through the
//                   nonlinear weights, tau, beta and the sub-stencil values
//   k_vjp_tpp       TPP: the same for the linear reconstruction (separable)
//   k_vjp_gather    cotangent of every padded cell (interior and ghost)
//                   (on large grids these run on groups of variables whose
//                   stencil cotangents fit in the space of the point values,
//                   no longer read; on small ones once for all three)
//   k_vjp_interior  the interior cotangent
//   k_vjp_ghost_t   plus G^T times the ghost cotangents (k_vjp_ghost_t_lds: by
//                   blocks of cells, the ghost cotangents they read staged in LDS,
//                   the blocks ordered by the canonical value records they read)
// Every kernel gathers (each output is written by one thread): no atomics.
// Scratch arrays are structs of arrays over cells, so that neighbouring lanes
// (neighbouring cells) read and write neighbouring addresses.
// Non-smooth points take the subgradient sign(0) = 0.
#include <type_traits>

#include "device_common.hpp"
#include "vjp_internal.hpp"

namespace hope {

// ---------------------------------------------------------------------------
// Adjoint helpers
// ---------------------------------------------------------------------------
// reverse mode of lmars(): given mu = dL/dF, accumulate dL/dqL and dL/dqR
// (TOPO: the pressure of phi* + phi_s, phi_s = sps / sqrtG a constant)
template <bool TOPO = false>
__device__ __forceinline__ void lmars_adj(const double* qL, const double* qR, double X, double Y, double sqx,
                                          double sqy, int dir, double ia, const double* mu, double* bL,
                                          double* bR, double sps = 0.0) {
  const double ox = sqx * sqx, oy = sqy * sqy;
  const double d2 = fma(X, X, oy);
  const double dl = sqrt_g(d2);
  const double idl = rcp(dl);
  const double isg = d2 * dl * ia * ia * rcp(ox * oy);
  const double sgii = dl * ia * rcp(dir == 0 ? sqx : sqy);
  // normal momentum component (selects, not a dynamic index: keeps the arrays in registers)
  const double qLn = dir == 0 ? qL[1] : qL[2], qRn = dir == 0 ? qR[1] : qR[2];
  const double phiL = qL[0] * isg, phiR = qR[0] * isg;
  const double iL = rcp(qL[0] * sgii), iR = rcp(qR[0] * sgii);
  const double upL = qLn * iL, upR = qRn * iR;
  const double sL = sqrt_g(phiL), sR = sqrt_g(phiR);
  const double c = 0.5 * (sL + sR);
  const double ic = rcp(c);
  const double ms = 0.5 * (upL + upR - (phiR - phiL) * ic);
  const double ps = 0.5 * (phiL + phiR - c * (upR - upL));
  const double mm = ms * sgii;
  const double am = fabs(mm);
  const double sg = mm > 0.0 ? 1.0 : (mm < 0.0 ? -1.0 : 0.0);
  // F_v = 1/2((mm + am) qL_v + (mm - am) qR_v) + pressure
  double mmb = 0.0, amb = 0.0;
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    bL[v] += 0.5 * (mm + am) * mu[v];
    bR[v] += 0.5 * (mm - am) * mu[v];
    mmb += 0.5 * (qL[v] + qR[v]) * mu[v];
    amb -= 0.5 * (qR[v] - qL[v]) * mu[v];
  }
  mmb += amb * sg;
  const double prb = dir == 0 ? mu[1] * oy + mu[2] * X * Y : mu[1] * X * Y + mu[2] * ox;
  const double psb = prb * (TOPO ? fma(sps, isg, ps) : ps) * idl;
  const double msb = mmb * sgii;
  double phiLb = 0.5 * psb, phiRb = 0.5 * psb;
  double cb = -0.5 * psb * (upR - upL);
  double upRb = -0.5 * psb * c, upLb = 0.5 * psb * c;
  upLb += 0.5 * msb;
  upRb += 0.5 * msb;
  phiRb -= 0.5 * msb * ic;
  phiLb += 0.5 * msb * ic;
  const double icb = -0.5 * msb * (phiR - phiL);
  cb -= icb * ic * ic;
  phiLb += 0.25 * cb * rcp(sL);
  phiRb += 0.25 * cb * rcp(sR);
  bL[1] += dir == 0 ? upLb * iL : 0.0;
  bL[2] += dir == 0 ? 0.0 : upLb * iL;
  bL[0] -= upLb * upL * (iL * sgii);        // upL / qL[0]
  bR[1] += dir == 0 ? upRb * iR : 0.0;
  bR[2] += dir == 0 ? 0.0 : upRb * iR;
  bR[0] -= upRb * upR * (iR * sgii);
  bL[0] += phiLb * isg;
  bR[0] += phiRb * isg;
}

// reverse mode of sources(): given (s1b, s2b) = dL/d(s1, s2), accumulate dL/dQ
__device__ __forceinline__ void sources_adj(double Q0, double Q1, double Q2, double X, double Y, double Lc,
                                            double omega2, double s1b, double s2b, double* Qb) {
  const double X2 = X * X, Y2 = Y * Y;
  const double id2 = rcp(1.0 + X2 + Y2);
  const double iq = 2.0 * rcp(Q0);
  const double A1 = Y * (1.0 + Y2) * Q1 * Q2 - X * Y2 * Q1 * Q1;
  const double A2 = X * (1.0 + X2) * Q1 * Q2 - X2 * Y * Q2 * Q2;
  const double f = omega2 * Lc;
  const double m1b = s1b * id2, c1b = s1b * id2, m2b = s2b * id2, c2b = s2b * id2;
  Qb[1] += c1b * (-f * X * Y) + c2b * (-f * (1.0 + X2));
  Qb[2] += c1b * (f * (1.0 + Y2)) + c2b * (f * X * Y);
  const double iqb = m1b * A1 + m2b * A2;
  const double A1b = m1b * iq, A2b = m2b * iq;
  Qb[1] += A1b * (Y * (1.0 + Y2) * Q2 - 2.0 * X * Y2 * Q1) + A2b * (X * (1.0 + X2) * Q2);
  Qb[2] += A1b * (Y * (1.0 + Y2) * Q1) + A2b * (X * (1.0 + X2) * Q1 - 2.0 * X2 * Y * Q2);
  Qb[0] -= iqb * iq * iq * 0.5;
}

// point number of side sd (0 left, 1 right, 2 bottom, 3 top), Gauss node h
template <int M>
__device__ __forceinline__ int side_pt(int sd, int h) { return sd * M + h; }

// ---------------------------------------------------------------------------
// k_vjp_traces: T[(pt*3 + v)*cells + c], one lane per (variable, cell) (struct of arrays: lanes of
// neighbouring cells touch neighbouring addresses)
// ---------------------------------------------------------------------------
template <int K, bool W, int M, bool TP>
__global__ __launch_bounds__(64) void k_vjp_traces(const double* __restrict__ tab_, GridScalars gs,
                                                    const double* __restrict__ q, double* __restrict__ T,
                                                    TopoDev tp) {
  using C = Cfg<K, W, M>;
  constexpr int NP = 4 * M + M * M;
  const cdp tab = (cdp)tab_;
  const int n = gs.n, P = gs.P;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 18 * n * n) return;
  const int cells_i = 6 * n * n;
  const int v = idx / cells_i, c = idx % cells_i;   // one lane per (variable, cell)
  const int p = c / (n * n), j = (c / n) % n, i = c % n;
  const size_t vs = (size_t)6 * P * P;
  const size_t coff = (size_t)p * P * P + (size_t)(j + C::R) * P + (i + C::R);
  const double* c0 = q + coff;
  // topography: the mass is reconstructed as sqrtG phi_t (cell averages of
  // sqrtG phi_s added), and each point value stored is the layer's own
  // sqrtG phi, as the forward stage kernel computes it
  const double* s0 = TP ? tp.sbar + coff : nullptr;
  const bool topo_v = TP && v == 0;
  const size_t cells = (size_t)cells_i;
  double* out = T + c;
  // the lane's stencil of one variable, staged in LDS: all its loads are
  // issued together instead of one by one inside the arithmetic
  constexpr bool kStage = K * K * 64 * 8 <= 32768;
  __shared__ double st[kStage ? K * K : 1][64];
  const int lane = threadIdx.x;
  {
    if constexpr (kStage) {
#pragma unroll
      for (int o = 0; o < K * K; ++o) {
        const int off = (o / K - C::R) * P + (o % K - C::R);
        st[o][lane] = c0[v * vs + off] + (topo_v ? s0[off] : 0.0);
      }
    }
    auto at = [&](int dy, int dx) -> double {
      if constexpr (kStage) return st[(dy + C::R) * K + dx + C::R][lane];
      else return c0[v * vs + dy * P + dx] + (topo_v ? s0[dy * P + dx] : 0.0);
    };
    auto sub = [&](double val, auto s_of) -> double {
      if constexpr (TP) return topo_v ? val - s_of() : val;
      else return val;
    };
    double kap[W ? C::S : 1];
    if constexpr (W) weno_kappa<K, W, M>(tab, gs.eps, at, [&](int jj, double x) { kap[jj] = x; });
    auto kf = [&](int jj) -> double { return kap[jj]; };
    double xr[C::XR];
    // a point's value as the forward computes it (WENO by columns)
    auto column = [&](int px, auto&& emit) {
      xpass<K, W, M>(tab, px, at, xr);
      if constexpr (W) {
        WCol<K, M> col;
        wcol<K, W, M>(tab, px, xr, kf, col);
        emit([&](int py, int pt) { return wpoint<K, W, M>(tab, px, py, pt, col); });
      } else {
        emit([&](int py, int pt) { return point<K, W, M>(tab, py, pt, xr, kf); });
      }
    };
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
      column(sd, [&](auto val) {
#pragma unroll
        for (int h = 0; h < M; ++h)
          out[((sd * M + h) * 3 + v) * cells] =
              sub(val(2 + h, sd * M + h), [&] { return topo_cell_side<M>(tp, n, p, i, j, sd, h); });
      });
#pragma unroll 1
    for (int h = 0; h < M; ++h)
      column(2 + h, [&](auto val) {
        out[((2 * M + h) * 3 + v) * cells] = sub(val(0, 2 * M + h), [&] { return topo_cell_side<M>(tp, n, p, i, j, 2, h); });
        out[((3 * M + h) * 3 + v) * cells] = sub(val(1, 3 * M + h), [&] { return topo_cell_side<M>(tp, n, p, i, j, 3, h); });
#pragma unroll
        for (int w = 0; w < M; ++w)
          out[((4 * M + w * M + h) * 3 + v) * cells] = sub(val(2 + w, 4 * M + w * M + h), [&] {
            return tp.sc[((((size_t)p * n + j) * n + i) * M + w) * M + h];
          });
      });
  }
}

// the converted neighbour trace at panel side sd, position t, Gauss node h of panel p
// (topography: the converted sqrtG phi_t, B's stored sqrtG phi plus its
// sqrtG phi_s, less sqrtG phi_s at this panel's point, as the forward forms it)
template <int M, bool TP = false>
__device__ __forceinline__ void outside_state(cdp tab, cip itab, const TabOffsets& O, int n, int P, int r,
                                              const double* __restrict__ T, int p, int sd, int t, int h,
                                              double* out, cdp* conv, int* bcell, int* bpt,
                                              const TopoDev& tp = TopoDev()) {
  constexpr int NP = 4 * M + M * M;
  const int idx = (p * 4 + sd) * n + t;
  const int off = itab[O.i_cell + idx];
  const int B = off / (P * P), jb = (off / P) % P - r, ib = off % P - r;
  const int bs = itab[O.i_side + idx];
  const int hb = itab[O.i_rev + idx] ? M - 1 - h : h;
  const int cb = (B * n + jb) * n + ib;
  const int pt = bs * M + hb;
  const size_t cells = (size_t)6 * n * n;
  const double* src = T + (size_t)pt * 3 * cells + cb;
  cdp cv = tab + O.bt_conv + ((size_t)idx * M + h) * 5;
  if constexpr (TP)
    out[0] = cv[0] * (src[0] + topo_cell_side<M>(tp, n, B, ib, jb, bs, hb)) - topo_side_point<M>(tp, n, idx, h);
  else
    out[0] = cv[0] * src[0];
  out[1] = cv[1] * src[cells] + cv[2] * src[2 * cells];
  out[2] = cv[3] * src[cells] + cv[4] * src[2 * cells];
  *conv = cv;
  *bcell = cb;
  *bpt = pt;
}

// ---------------------------------------------------------------------------
// k_vjp_points: Lam[(pt*3 + v)*cells + c] = dL/d(point value).  Lanes
// [0, 12 n (n+1)) take one cell edge each (panel p, direction, position):
// the flux adjoint at its m Gauss points gives the cotangents of both
// traces, written to the edge points of the cells on either side (a panel
// edge's outside trace belongs to the neighbour panel and is handled by
// k_vjp_edges).  Each point slot has exactly one writer.  The remaining
// 6 n^2 lanes take one cell each: the source adjoint at its m^2 nodes.
// ---------------------------------------------------------------------------
template <int K, bool W, int M, bool TP>
__global__ __launch_bounds__(64) void k_vjp_points(const double* __restrict__ tab_, const int32_t* __restrict__ itab_,
                                                    GridScalars gs, const double* __restrict__ T,
                                                    const double* __restrict__ w, double* __restrict__ Lam,
                                                    TopoDev tp, double* __restrict__ Lder) {
  using C = Cfg<K, W, M>;
  const cdp tab = (cdp)tab_;
  const cip itab = (cip)itab_;
  const int n = gs.n, P = gs.P;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int edges = 12 * n * (n + 1);
  if (t >= edges + 6 * n * n) return;
  const TabOffsets O = tab_offsets(K, W, M, n);
  const double invd = gs.inv_delta, ia = 1.0 / gs.radius;
  const size_t nn = (size_t)n * n;
  const size_t cells = (size_t)6 * n * n;
  auto wv = [&](int v, int cc) -> double { return w[(size_t)v * 6 * nn + cc]; };
  auto tr = [&](int pt, int v, int cc) -> double { return T[((size_t)pt * 3 + v) * cells + cc]; };
  auto lam = [&](int pt, int v, int cc) -> double& { return Lam[((size_t)pt * 3 + v) * cells + cc]; };
  cdp Xg = tab + O.Xg, sqg = tab + O.sqg, Xe = tab + O.Xe, sqe = tab + O.sqe, gw = tab + C::O.gw;
  if (t < edges) {
    const int per = (n + 1) * n;
    const int pd = t / per, loc = t % per;
    const int p = pd >> 1, dir = pd & 1;
    // x edge e between cells (e-1, a) and (e, a); y edge e between (a, e-1) and (a, e)
    const int e = dir == 0 ? loc % (n + 1) : loc / n;
    const int a = dir == 0 ? loc / (n + 1) : loc % n;
    const bool inL = e > 0, inR = e < n;
    const int cL = dir == 0 ? (p * n + a) * n + (e - 1) : (p * n + (e - 1)) * n + a;
    const int cR = dir == 0 ? (p * n + a) * n + e : (p * n + e) * n + a;
    const int sdL = dir == 0 ? 1 : 3, sdR = dir == 0 ? 0 : 2;   // the edge's side in each cell
    // the flux through the edge adds +F/D to the right (top) cell and -F/D to the other
    double dF[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) dF[v] = ((inR ? wv(v, cR) : 0.0) - (inL ? wv(v, cL) : 0.0)) * invd;
#pragma unroll
    for (int h = 0; h < M; ++h) {
      double qL[3], qR[3];
      cdp cv;
      int bc, bp;
      if (inL) {
#pragma unroll
        for (int v = 0; v < 3; ++v) qL[v] = tr(sdL * M + h, v, cL);
      } else {
        outside_state<M, TP>(tab, itab, O, n, P, gs.r, T, p, sdR, a, h, qL, &cv, &bc, &bp, tp);
      }
      if (inR) {
#pragma unroll
        for (int v = 0; v < 3; ++v) qR[v] = tr(sdR * M + h, v, cR);
      } else {
        outside_state<M, TP>(tab, itab, O, n, P, gs.r, T, p, sdL, a, h, qR, &cv, &bc, &bp, tp);
      }
      double X, Y, sx, sy;
      if (dir == 0) { X = Xe[e]; sx = sqe[e]; Y = Xg[a * M + h]; sy = sqg[a * M + h]; }
      else { X = Xg[a * M + h]; sx = sqg[a * M + h]; Y = Xe[e]; sy = sqe[e]; }
      double mu[3] = {gw[h] * dF[0], gw[h] * dF[1], gw[h] * dF[2]};
      double bL[3] = {0, 0, 0}, bR[3] = {0, 0, 0};
      double sps = 0.0;
      if constexpr (TP)
        sps = dir == 0 ? tp.sx[(((size_t)p * n + a) * (n + 1) + e) * M + h]
                       : tp.sy[(((size_t)p * (n + 1) + e) * n + a) * M + h];
      lmars_adj<TP>(qL, qR, X, Y, sx, sy, dir, ia, mu, bL, bR, sps);
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        if (inL) lam(sdL * M + h, v, cL) = bL[v];
        if (inR) lam(sdR * M + h, v, cR) = bR[v];
      }
    }
    return;
  }
  // sources at the cell Gauss points
  const int c = t - edges;
  const int p = c / (n * n), j = (c / n) % n, i = c % n;
  cdp fc = tab + C::O.fcoef + p * 3;
#pragma unroll
  for (int vv = 0; vv < M; ++vv)
#pragma unroll
    for (int h = 0; h < M; ++h) {
      const int pt = 4 * M + vv * M + h;
      const double X = Xg[i * M + h], Y = Xg[j * M + vv];
      const double g2 = gw[h] * gw[vv];
      double Qb[3] = {0, 0, 0};
      sources_adj(tr(pt, 0, c), tr(pt, 1, c), tr(pt, 2, c), X, Y, fc[0] + fc[1] * X + fc[2] * Y,
                  gs.omega2, g2 * wv(1, c), g2 * wv(2, c), Qb);
      if constexpr (TP) {
        // psi_B (2.14) is linear in sqrtG phi_t at the node and its two
        // derivatives; the latter's cotangents go to Lder for the stencil adjoint
        double Tb, Txib, Tetab;
        psi_b_adj(X, Y, tp.sc[((((size_t)p * n + j) * n + i) * M + vv) * M + h], invd, ia, g2 * wv(1, c),
                  g2 * wv(2, c), Tb, Txib, Tetab);
        Qb[0] += Tb;
        Lder[((size_t)(vv * M + h)) * cells + c] = Txib;
        Lder[((size_t)(M * M + vv * M + h)) * cells + c] = Tetab;
      }
#pragma unroll
      for (int v = 0; v < 3; ++v) lam(pt, v, c) = Qb[v];
    }
}

// ---------------------------------------------------------------------------
// k_vjp_edges: the neighbour panel's flux at its edge points, adjoint w.r.t.
// the converted trace, added to the owning cell's point cotangent
// ---------------------------------------------------------------------------
template <int K, bool W, int M, bool TP>
__global__ __launch_bounds__(64) void k_vjp_edges(const double* __restrict__ tab_, const int32_t* __restrict__ itab_,
                                                   GridScalars gs, const double* __restrict__ T,
                                                   const double* __restrict__ w, double* __restrict__ Lam,
                                                   TopoDev tp) {
  using C = Cfg<K, W, M>;
  constexpr int NP = 4 * M + M * M;
  const cdp tab = (cdp)tab_;
  const cip itab = (cip)itab_;
  const int n = gs.n, P = gs.P;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 24 * n * M) return;
  const TabOffsets O = tab_offsets(K, W, M, n);
  const int h = k % M;
  const int t = (k / M) % n;
  const int sd = (k / (M * n)) % 4;
  const int p = k / (M * n * 4);
  const int i = sd == 0 ? 0 : sd == 1 ? n - 1 : t;
  const int j = sd == 2 ? 0 : sd == 3 ? n - 1 : t;
  const int c = (p * n + j) * n + i;
  const size_t nn = (size_t)n * n;
  const double invd = gs.inv_delta, ia = 1.0 / gs.radius;
  cdp Xg = tab + O.Xg, sqg = tab + O.sqg, Xe = tab + O.Xe, sqe = tab + O.sqe, gw = tab + C::O.gw;
  double qo[3], qn[3];
#pragma unroll
  for (int v = 0; v < 3; ++v) qo[v] = T[((size_t)(sd * M + h) * 3 + v) * nn * 6 + c];
  cdp cv;
  int bc, bp;
  outside_state<M, TP>(tab, itab, O, n, P, gs.r, T, p, sd, t, h, qn, &cv, &bc, &bp, tp);
  const bool own_is_right = (sd == 0 || sd == 2);
  const int dir = sd < 2 ? 0 : 1;
  const int e = sd == 0 ? 0 : sd == 1 ? n : sd == 2 ? 0 : n;
  double X, Y, sx, sy;
  if (dir == 0) { X = Xe[e]; sx = sqe[e]; Y = Xg[j * M + h]; sy = sqg[j * M + h]; }
  else { X = Xg[i * M + h]; sx = sqg[i * M + h]; Y = Xe[e]; sy = sqe[e]; }
  double mu[3];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const double wc = w[(size_t)v * 6 * nn + c];
    mu[v] = gw[h] * (own_is_right ? wc : -wc) * invd;
  }
  double bL[3] = {0, 0, 0}, bR[3] = {0, 0, 0};
  const double sps = TP ? topo_side_point<M>(tp, n, (p * 4 + sd) * n + t, h) : 0.0;
  if (own_is_right) lmars_adj<TP>(qn, qo, X, Y, sx, sy, dir, ia, mu, bL, bR, sps);
  else lmars_adj<TP>(qo, qn, X, Y, sx, sy, dir, ia, mu, bL, bR, sps);
  double ob[3];                                   // cotangent of the converted outside state
#pragma unroll
  for (int v = 0; v < 3; ++v) ob[v] = own_is_right ? bL[v] : bR[v];
  const size_t cells = 6 * nn;
  double* dst = Lam + (size_t)bp * 3 * cells + bc;
  dst[0] += cv[0] * ob[0];
  dst[cells] += cv[1] * ob[1] + cv[3] * ob[2];
  dst[2 * cells] += cv[2] * ob[1] + cv[4] * ob[2];
}

// ---------------------------------------------------------------------------
// k_vjp_weno: Dl[(o*3 + v)*cells + c] = cotangent of stencil cell o of cell c
// ---------------------------------------------------------------------------
// topography: the cotangents Lder of d(sqrtG phi_t)/dxi and /deta at the
// cell nodes (psi_B of (2.14)) reach the mass stencil through the centred
// derivative weights, d/dxi = sum_b wc_y[b] sum_a wd_x[a] q[b][a] and
// d/deta = sum_b wd_y[b] sum_a wc_x[a] q[b][a] at x node h, y node w
// one stencil row: add(col, x) for its K cells; ld(k) = Lder[k * cells + c]
template <int K, int M, typename Ld, typename Add>
__device__ __forceinline__ void topo_row_adj(cdp tab, Ld ld, int row, Add add) {
  using C = Cfg<K, false, M>;
  cdp wc = tab + C::O.wc, wd = tab + C::O.wd;
  double ya[M], yb[M];
#pragma unroll
  for (int h = 0; h < M; ++h) {
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int w = 0; w < M; ++w) {
      sa = fma(ld(w * M + h), wc[(2 + w) * K + row], sa);
      sb = fma(ld(M * M + w * M + h), wd[(2 + w) * K + row], sb);
    }
    ya[h] = sa;
    yb[h] = sb;
  }
#pragma unroll
  for (int col = 0; col < K; ++col) {
    double s = 0.0;
#pragma unroll
    for (int h = 0; h < M; ++h) s = fma(ya[h], wd[(2 + h) * K + col], fma(yb[h], wc[(2 + h) * K + col], s));
    add(col, s);
  }
}

template <int K, int M, typename Add>
__device__ __forceinline__ void topo_derivative_adj(cdp tab, const double* __restrict__ Lder, size_t cells, int c,
                                                    Add add) {
  auto ld = [&](int k) -> double { return Lder[(size_t)k * cells + c]; };
#pragma unroll 1
  for (int row = 0; row < K; ++row) topo_row_adj<K, M>(tab, ld, row, [&](int col, double x) { add(row * K + col, x); });
}

// ---------------------------------------------------------------------------
// Adjoint of the genuine 2D WENO reconstruction (3.16)-(3.25) of one variable
// of one cell: at(dy, dx) is the stencil, lamf(pt) the cotangent of point pt's
// value; the cotangents of the K x K stencil cells are accumulated into
// dq(o), o = (dy + R) K + dx + R (zero on entry).  Shared by the per-cell
// kernel and the marching kernel, so both give the same values bit for bit.
// ---------------------------------------------------------------------------
template <int K, bool W, int M, typename At, typename LamF, typename Dq>
__device__ __forceinline__ void weno_cell_adj(cdp tab, double eps, At at, LamF lamf, Dq dq) {
  using C = Cfg<K, W, M>;
  constexpr int R = C::R, L = C::L, S = C::S, NR = C::NR, NA = C::NA;
  (void)R;
  cdp V = tab + C::O.V, lamq = tab + C::O.lam, wsub = tab + C::O.wsub;
  // forward smoothness indicators
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
          double cc = 0;
#pragma unroll
          for (int bb = 0; bb < L; ++bb) cc = fma(V[(sy * L + be) * L + bb], tr[sy + bb][al], cc);
          b = fma(lamq[be * L + al] * cc, cc, b);
        }
      beta[sy * L + sx] = b;
    }
  }
  double tau = 0;
#pragma unroll
  for (int a = 0; a < S; ++a)
#pragma unroll
    for (int b = a + 1; b < S; ++b) tau += fabs(beta[a] - beta[b]);
  const double ctau = 2.0 / (S * (S + 1));
  tau *= ctau;
  double kap[S], kapb[S];
#pragma unroll
  for (int jj = 0; jj < S; ++jj) {
    kap[jj] = fma(tau, rcp(beta[jj] + eps), 1.0);
    kapb[jj] = 0.0;
  }
  // points, grouped by their x axis point px, evaluated by columns as the
  // forward does (wcol / wpoint): per column Z[sy][b] = sum_sx e[sy][sx]
  // xr[sx][sy+b] and E[sy] = sum_sx e[sy][sx] with e = d_sx kappa (and the
  // |d_sx| versions Za, Ea for the centre node); per point B, D (and A, C)
  cdp d1 = tab + C::O.d1;
  const double th = tab[C::O.theta];
  // one x axis point; the mixed-sign centre node (xm) keeps the abs(d)
  // column sums as well, the other nodes are compiled without them
  auto column_pass = [&](auto mixed, int px) {
    constexpr bool xm = decltype(mixed)::value;
    double xr[L * NR];
#pragma unroll
    for (int sx = 0; sx < L; ++sx)
#pragma unroll
      for (int row = 0; row < NR; ++row) {
        double s = 0;
#pragma unroll
        for (int a = 0; a < L; ++a) s = fma(wsub[(sx * NA + px) * L + a], at(row - R, sx - (L - 1) + a), s);
        xr[sx * NR + row] = s;
      }
    double e[L][L], E[L], Z[L][L], ea[L][L], Ea[L], Za[L][L];
    double Zb[L][L], Eb[L], Zab[L][L], Eab[L];
#pragma unroll
    for (int sy = 0; sy < L; ++sy) {
      E[sy] = 0.0;
      Ea[sy] = 0.0;
      Eb[sy] = 0.0;
      Eab[sy] = 0.0;
#pragma unroll
      for (int sx = 0; sx < L; ++sx) {
        e[sy][sx] = d1[px * L + sx] * kap[sy * L + sx];
        E[sy] += e[sy][sx];
        if (xm) {
          ea[sy][sx] = fabs(d1[px * L + sx]) * kap[sy * L + sx];
          Ea[sy] += ea[sy][sx];
        }
      }
#pragma unroll
      for (int b = 0; b < L; ++b) {
        double z = 0.0, za = 0.0;
#pragma unroll
        for (int sx = 0; sx < L; ++sx) {
          z = fma(e[sy][sx], xr[sx * NR + sy + b], z);
          if (xm) za = fma(ea[sy][sx], xr[sx * NR + sy + b], za);
        }
        Z[sy][b] = z;
        Za[sy][b] = za;
        Zb[sy][b] = 0.0;
        Zab[sy][b] = 0.0;
      }
    }
    const int npy = px < 2 ? M : M + 2;
#pragma unroll
    for (int k = 0; k < npy; ++k) {
      int py, pt;
      if (px < 2) { py = 2 + k; pt = px * M + k; }
      else {
        const int h = px - 2;
        if (k == 0) { py = 0; pt = 2 * M + h; }
        else if (k == 1) { py = 1; pt = 3 * M + h; }
        else { py = k; pt = 4 * M + (k - 2) * M + h; }
      }
      const bool ym = weno_mixed_axis(K, M, py);
      const double lb = lamf(pt);
      // forward of the point
      double T[L], Ta[L];
      double B = 0.0, D = 0.0, A = 0.0, Cs = 0.0;
#pragma unroll
      for (int sy = 0; sy < L; ++sy) {
        double t = 0.0, ta = 0.0;
#pragma unroll
        for (int b = 0; b < L; ++b) {
          t = fma(wsub[(sy * NA + py) * L + b], Z[sy][b], t);
          if (xm) ta = fma(wsub[(sy * NA + py) * L + b], Za[sy][b], ta);
        }
        T[sy] = t;
        Ta[sy] = ta;
        const double dy = d1[py * L + sy];
        B = fma(dy, t, B);
        D = fma(dy, E[sy], D);
        if (xm) {
          A = fma(fabs(dy), ta, A);
          Cs = fma(fabs(dy), Ea[sy], Cs);
        } else if (ym) {
          A = fma(fabs(dy), t, A);
          Cs = fma(fabs(dy), E[sy], Cs);
        }
      }
      // adjoint of the value: cotangents of B, D, A, C
      double Bb, Db, Ab = 0.0, Cb = 0.0;
      if (!xm && !ym) {
        const double iD = rcp(D);
        Bb = lb * iD;
        Db = -Bb * B * iD;
      } else {
        const double N1 = fma(th, A, B), D1 = fma(th, Cs, D), N2 = fma(th, A, -B), D2 = fma(th, Cs, -D);
        const double i1 = rcp(D1), i2 = rcp(D2);
        const double sp = tab[C::O.sp + pt], sm = tab[C::O.sm + pt];
        const double N1b = sp * lb * i1, D1b = -N1b * N1 * i1;
        const double N2b = -sm * lb * i2, D2b = -N2b * N2 * i2;
        Ab = th * (N1b + N2b);
        Bb = N1b - N2b;
        Cb = th * (D1b + D2b);
        Db = D1b - D2b;
      }
      // back to the column sums
#pragma unroll
      for (int sy = 0; sy < L; ++sy) {
        const double dy = d1[py * L + sy];
        double Tb = dy * Bb;
        Eb[sy] = fma(dy, Db, Eb[sy]);
        if (xm) {
          const double Tab = fabs(dy) * Ab;
          Eab[sy] = fma(fabs(dy), Cb, Eab[sy]);
#pragma unroll
          for (int b = 0; b < L; ++b) Zab[sy][b] = fma(wsub[(sy * NA + py) * L + b], Tab, Zab[sy][b]);
        } else if (ym) {
          Tb = fma(fabs(dy), Ab, Tb);
          Eb[sy] = fma(fabs(dy), Cb, Eb[sy]);
        }
#pragma unroll
        for (int b = 0; b < L; ++b) Zb[sy][b] = fma(wsub[(sy * NA + py) * L + b], Tb, Zb[sy][b]);
      }
    }
    // column adjoint: to kappa (through e = d kappa) and to the x-pass
    double xrb[L * NR];
#pragma unroll
    for (int o = 0; o < L * NR; ++o) xrb[o] = 0.0;
#pragma unroll
    for (int sy = 0; sy < L; ++sy)
#pragma unroll
      for (int sx = 0; sx < L; ++sx) {
        double eb = Eb[sy];
#pragma unroll
        for (int b = 0; b < L; ++b) {
          eb = fma(Zb[sy][b], xr[sx * NR + sy + b], eb);
          xrb[sx * NR + sy + b] = fma(e[sy][sx], Zb[sy][b], xrb[sx * NR + sy + b]);
        }
        kapb[sy * L + sx] = fma(d1[px * L + sx], eb, kapb[sy * L + sx]);
        if (xm) {
          double eab = Eab[sy];
#pragma unroll
          for (int b = 0; b < L; ++b) {
            eab = fma(Zab[sy][b], xr[sx * NR + sy + b], eab);
            xrb[sx * NR + sy + b] = fma(ea[sy][sx], Zab[sy][b], xrb[sx * NR + sy + b]);
          }
          kapb[sy * L + sx] = fma(fabs(d1[px * L + sx]), eab, kapb[sy * L + sx]);
        }
      }
    // x-pass adjoint
#pragma unroll
    for (int sx = 0; sx < L; ++sx)
#pragma unroll
      for (int row = 0; row < NR; ++row)
#pragma unroll
        for (int a = 0; a < L; ++a)
          dq(row * K + (sx + a)) = fma(wsub[(sx * NA + px) * L + a], xrb[sx * NR + row], dq(row * K + (sx + a)));
  };
#pragma unroll 1
  for (int px = 0; px < NA; ++px) {
    if (weno_mixed_axis(K, M, px)) column_pass(std::true_type{}, px);
    else column_pass(std::false_type{}, px);
  }
  // kappa_j = 1 + tau/(beta_j + eps)
  double taub = 0, betab[S];
#pragma unroll
  for (int jj = 0; jj < S; ++jj) {
    const double ib = rcp(beta[jj] + eps);
    taub += kapb[jj] * ib;
    betab[jj] = -kapb[jj] * tau * ib * ib;
  }
#pragma unroll
  for (int a = 0; a < S; ++a)
#pragma unroll
    for (int b = a + 1; b < S; ++b) {
      const double d = beta[a] - beta[b];
      const double sg = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
      betab[a] += taub * ctau * sg;
      betab[b] -= taub * ctau * sg;
    }
  // beta_j = sum lam c^2, c = (V_sy x V_sx) q
#pragma unroll
  for (int sx = 0; sx < L; ++sx) {
    double tr[NR][L], trb[NR][L];
#pragma unroll
    for (int row = 0; row < NR; ++row)
#pragma unroll
      for (int al = 0; al < L; ++al) {
        double s = 0;
#pragma unroll
        for (int a = 0; a < L; ++a) s = fma(V[(sx * L + al) * L + a], at(row - R, sx - (L - 1) + a), s);
        tr[row][al] = s;
        trb[row][al] = 0.0;
      }
#pragma unroll
    for (int sy = 0; sy < L; ++sy) {
      const double bb_ = betab[sy * L + sx];
#pragma unroll
      for (int be = 0; be < L; ++be)
#pragma unroll
        for (int al = 0; al < L; ++al) {
          if (al == 0 && be == 0) continue;
          double cc = 0;
#pragma unroll
          for (int bb = 0; bb < L; ++bb) cc = fma(V[(sy * L + be) * L + bb], tr[sy + bb][al], cc);
          const double ccb = 2.0 * lamq[be * L + al] * cc * bb_;
#pragma unroll
          for (int bb = 0; bb < L; ++bb) trb[sy + bb][al] += V[(sy * L + be) * L + bb] * ccb;
        }
    }
#pragma unroll
    for (int row = 0; row < NR; ++row)
#pragma unroll
      for (int al = 0; al < L; ++al)
#pragma unroll
        for (int a = 0; a < L; ++a) dq(row * K + (sx + a)) += V[(sx * L + al) * L + a] * trb[row][al];
  }
}

template <int K, bool W, int M, bool TP>
__global__ __launch_bounds__(64) void k_vjp_weno(const double* __restrict__ tab_, GridScalars gs,
                                                  const double* __restrict__ q, const double* __restrict__ Lam,
                                                  double* __restrict__ Dl, TopoDev tp,
                                                  const double* __restrict__ Lder, int v0, int nv) {
  using C = Cfg<K, W, M>;
  constexpr int NP = 4 * M + M * M, R = C::R;
  const cdp tab = (cdp)tab_;
  const int n = gs.n, P = gs.P;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int cells = 6 * n * n;
  if (idx >= nv * cells) return;
  // variables v0 .. v0+nv-1; stencil cotangents [K^2][nv][cells]
  const int v = v0 + idx / cells, c = idx % cells;
  const size_t dl_stride = (size_t)nv * cells;
  const int p = c / (n * n), j = (c / n) % n, i = c % n;
  const size_t vs = (size_t)6 * P * P;
  const size_t coff = (size_t)p * P * P + (size_t)(j + R) * P + (i + R);
  const double* c0 = q + v * vs + coff;
  // the lane's stencil, staged in LDS (see k_vjp_traces); with topography
  // the mass stencil is that of sqrtG phi_t
  __shared__ double st[K * K][64];
  __shared__ double sl[NP][64];
  const int lane = threadIdx.x;
  const bool topo_v = TP && v == 0;
#pragma unroll
  for (int o = 0; o < K * K; ++o) {
    const int off = (o / K - R) * P + (o % K - R);
    st[o][lane] = c0[off] + (topo_v ? tp.sbar[coff + off] : 0.0);
  }
  auto at = [&](int dy, int dx) -> double { return st[(dy + R) * K + dx + R][lane]; };
  {
    const double* lam = Lam + (size_t)v * cells + c;     // point pt at lam[pt * 3 * cells]
#pragma unroll
    for (int pt = 0; pt < NP; ++pt) sl[pt][lane] = lam[(size_t)pt * 3 * cells];
  }
  double dq[K * K];
#pragma unroll
  for (int o = 0; o < K * K; ++o) dq[o] = 0.0;
  weno_cell_adj<K, W, M>(tab, gs.eps, at, [&](int pt) -> double { return sl[pt][lane]; },
                         [&](int o) -> double& { return dq[o]; });
  if constexpr (TP) {
    if (v == 0) topo_derivative_adj<K, M>(tab, Lder, cells, c, [&](int o, double x) { dq[o] += x; });
  }
  double* out = Dl + (size_t)(v - v0) * cells + c;
#pragma unroll
  for (int o = 0; o < K * K; ++o) out[(size_t)o * dl_stride] = dq[o];
}

// ---------------------------------------------------------------------------
// Adjoint of the TPP (linear) reconstruction of one variable of one cell, one
// stencil row at a time: a point value is wy[py] (x) wx[px] applied to the
// stencil, so the cotangent of stencil cell (row, col) is the sum over points
// of lam_pt wc[py][row] wc[px][col]: first the y-sums for each x axis point,
// then the x-sums.  emit(col, x) for the K cells of the row.
// ---------------------------------------------------------------------------
template <int K, bool W, int M, typename LamF, typename Emit>
__device__ __forceinline__ void tpp_row_adj(cdp tab, LamF L, int row, Emit emit) {
  using C = Cfg<K, W, M>;
  constexpr int NA = C::NA;
  cdp wc = tab + C::O.wc;
  double yr[NA];
#pragma unroll
  for (int px = 0; px < 2; ++px) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < M; ++k) s = fma(L(px * M + k), wc[(2 + k) * K + row], s);
    yr[px] = s;
  }
#pragma unroll
  for (int h = 0; h < M; ++h) {
    double s = L(2 * M + h) * wc[0 * K + row];
    s = fma(L(3 * M + h), wc[1 * K + row], s);
#pragma unroll
    for (int w = 0; w < M; ++w) s = fma(L(4 * M + w * M + h), wc[(2 + w) * K + row], s);
    yr[2 + h] = s;
  }
#pragma unroll
  for (int col = 0; col < K; ++col) {
    double s = 0.0;
#pragma unroll
    for (int px = 0; px < NA; ++px) s = fma(yr[px], wc[px * K + col], s);
    emit(col, s);
  }
}

// ---------------------------------------------------------------------------
// k_vjp_tpp: TPP (linear) reconstruction adjoint, Dl as in k_vjp_weno
// ---------------------------------------------------------------------------
template <int K, bool W, int M, bool TP>
__global__ __launch_bounds__(64) void k_vjp_tpp(const double* __restrict__ tab_, GridScalars gs,
                                                 const double* __restrict__ Lam, double* __restrict__ Dl,
                                                 const double* __restrict__ Lder, int v0, int nv) {
  const cdp tab = (cdp)tab_;
  const int n = gs.n;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int cells = 6 * n * n;
  if (idx >= nv * cells) return;
  const int v = v0 + idx / cells, c = idx % cells;
  const size_t dl_stride = (size_t)nv * cells;
  const double* lam = Lam + (size_t)v * cells + c;     // point pt at lam[pt * 3 * cells]
  auto L = [&](int pt) -> double { return lam[(size_t)pt * 3 * cells]; };
  double* out = Dl + (size_t)(v - v0) * cells + c;
#pragma unroll 1
  for (int row = 0; row < K; ++row)
    tpp_row_adj<K, W, M>(tab, L, row, [&](int col, double x) { out[(size_t)(row * K + col) * dl_stride] = x; });
  if constexpr (TP) {
    if (v == 0)
      topo_derivative_adj<K, M>(tab, Lder, (size_t)cells, c, [&](int o, double x) { out[(size_t)o * dl_stride] += x; });
  }
}

// ---------------------------------------------------------------------------
// k_vjp_gather: cotangent of padded cell (v, p, jj, ii) = sum of the stencil
// cotangents Dl of the cells whose stencil holds it
// ---------------------------------------------------------------------------
template <int K, bool W, int M>
__global__ __launch_bounds__(256) void k_vjp_gather(const double* __restrict__ tab_, GridScalars gs,
                                                     const double* __restrict__ Lam, const double* __restrict__ Dl,
                                                     double* __restrict__ gpad, int v0, int nv) {
  using C = Cfg<K, W, M>;
  constexpr int R = C::R;
  (void)tab_;
  (void)Lam;
  const int n = gs.n, P = gs.P;
  const size_t plane = (size_t)6 * P * P;              // one variable's padded plane
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nv * plane) return;
  const int v = v0 + (int)(idx / plane);
  const size_t pi = idx % plane;
  const int ii = pi % P, jj = (pi / P) % P, p = (int)(pi / ((size_t)P * P));
  const size_t cells = (size_t)6 * n * n;
  // a stencil row's K values are requested together (the cells outside the
  // panel masked), then added in the order of the row: the same sum as
  // adding the in-panel values one by one
  double acc = 0.0;
#pragma unroll(K <= 5 ? K : 1)
  for (int dy = -R; dy <= R; ++dy) {
    const int j = jj - R - dy;
    const bool jin = j >= 0 && j < n;
    double val[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const int i = ii - t;   // dx = t - R
      const bool in = jin && i >= 0 && i < n;
      const size_t o = (size_t)(dy + R) * K + t;
      val[t] = in ? Dl[(o * nv + (v - v0)) * cells + (size_t)(p * n + j) * n + i] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const int i = ii - t;
      if (jin && i >= 0 && i < n) acc += val[t];
    }
  }
  gpad[(size_t)v * plane + pi] = acc;
}

// ---------------------------------------------------------------------------
// k_vjp_interior: gq = the interior part of the padded cotangent
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_vjp_interior(int n, int P, int r, const double* __restrict__ gpad,
                                                      double* __restrict__ gq) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= 6 * n * n) return;
  const int p = c / (n * n), j = (c / n) % n, i = c % n;
  const size_t plane = (size_t)6 * P * P;
  const size_t off = (size_t)p * P * P + (size_t)(j + r) * P + (i + r);
  const size_t nn = (size_t)6 * n * n;
  gq[c] = gpad[off];
  gq[nn + c] = gpad[plane + off];
  gq[2 * nn + c] = gpad[2 * plane + off];
}

// ---------------------------------------------------------------------------
// k_vjp_ghost_t: gq += G^T (ghost cotangents), 16 lanes per interior cell
// that some ghost row reads (the only rows of G^T with entries)
// (c1, c2) -> T (c1, c2) for a frame code of the compressed ghost map: the
// image of panel coordinates (X, Y) is (sx (sw ? Y : X), sy (sw ? X : Y)),
// sw = f & 1, sx = -1 if f & 2, sy = -1 if f & 4
__device__ __forceinline__ void frame_apply_t(int f, double c1, double c2, double& g1, double& g2) {
  const bool sw = f & 1;
  const double sx = (f & 2) ? -1.0 : 1.0, sy = (f & 4) ? -1.0 : 1.0;
  g1 = sx * (sw ? c2 : c1);
  g2 = sy * (sw ? c1 : c2);
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_vjp_ghost_t(int rows, int n, int P, const int32_t* __restrict__ gt_cell,
                                                     const int32_t* __restrict__ gt_ptr,
                                                     const int32_t* __restrict__ gt_row,
                                                     const int32_t* __restrict__ gt_ref,
                                                     const GhostVal* __restrict__ gcval,
                                                     const double* __restrict__ gpad, double* __restrict__ gq) {
  const int row = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 4);
  if (row >= rows) return;   // whole 16-lane group leaves together
  const int lane = threadIdx.x & 15;
  const size_t plane = (size_t)6 * P * P;
  double g0 = 0.0, g1 = 0.0, g2 = 0.0;
  for (int k = gt_ptr[row] + lane; k < gt_ptr[row + 1]; k += 16) {
    const int d = gt_row[k];
    const double a0 = gpad[d], a1 = gpad[plane + d], a2 = gpad[2 * plane + d];
    // the G entry's momentum block T(f0) C T(f)^T from its canonical record
    // (signed permutations: exact, the values G applied in the forward fill)
    const int ref = gt_ref[k];
    const GhostVal cj = gcval[ref & 0xffffff];
    const int f = (ref >> 24) & 7, f0 = (ref >> 27) & 7;
    double m11, m12, m21, m22, b11, b12, b21, b22;
    frame_apply_t(f, cj.v[1], cj.v[2], m11, m12);
    frame_apply_t(f, cj.v[3], cj.v[4], m21, m22);
    frame_apply_t(f0, m11, m21, b11, b21);
    frame_apply_t(f0, m12, m22, b12, b22);
    g0 = fma(cj.v[0], a0, g0);
    g1 = fma(b11, a1, fma(b21, a2, g1));
    g2 = fma(b12, a1, fma(b22, a2, g2));
  }
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) {
    g0 += __shfl_xor(g0, off, 16);
    g1 += __shfl_xor(g1, off, 16);
    g2 += __shfl_xor(g2, off, 16);
  }
  if (lane == 0) {
    const int c = gt_cell[row];
    const size_t nn = (size_t)6 * n * n;
    gq[c] += g0;
    gq[nn + c] += g1;
    gq[2 * nn + c] += g2;
  }
}

// the same by blocks of kGtCells rows (block b: rows b kGtCells ..): the
// ghost cotangents the block reads are first copied to LDS (3 x umax), then
// each row's 16 lanes sum their entries from there, in the order above.  The
// blocks run in the order of the list border (by the canonical value records
// they read), each L2 domain a contiguous range of it, so that one domain
// reads a narrow band of the records instead of all of them
__global__ __launch_bounds__(256) void k_vjp_ghost_t_lds(int blocks, const int32_t* __restrict__ border,
                                                         int rows, int n, int P, int umax,
                                                         const int32_t* __restrict__ gt_cell,
                                                         const int32_t* __restrict__ gt_ptr,
                                                         const int32_t* __restrict__ gt_bptr,
                                                         const int32_t* __restrict__ gt_bsrc,
                                                         const uint16_t* __restrict__ gt_lidx,
                                                         const int32_t* __restrict__ gt_ref,
                                                         const GhostVal* __restrict__ gcval,
                                                         const double* __restrict__ gpad, double* __restrict__ gq) {
  extern __shared__ double sg[];
  // each L2 domain takes a contiguous range of the block list
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  if (lb >= blocks) return;   // the whole workgroup leaves together
  const int b = border[lb];
  const size_t plane = (size_t)6 * P * P;
  const int s0 = gt_bptr[b], U = gt_bptr[b + 1] - s0;
  for (int u = threadIdx.x; u < U; u += blockDim.x) {
    const int d = gt_bsrc[s0 + u];
    sg[u] = gpad[d];
    sg[umax + u] = gpad[plane + d];
    sg[2 * umax + u] = gpad[2 * plane + d];
  }
  __syncthreads();
  const int row = b * kGtCells + (int)threadIdx.x / 16;
  if (row >= rows) return;   // the whole 16-lane group leaves together
  const int lane = threadIdx.x & 15;
  double g0 = 0.0, g1 = 0.0, g2 = 0.0;
  for (int k = gt_ptr[row] + lane; k < gt_ptr[row + 1]; k += 16) {
    const int l = gt_lidx[k];
    const double a0 = sg[l], a1 = sg[umax + l], a2 = sg[2 * umax + l];
    const int ref = gt_ref[k];
    const GhostVal cj = gcval[ref & 0xffffff];
    const int f = (ref >> 24) & 7, f0 = (ref >> 27) & 7;
    double m11, m12, m21, m22, b11, b12, b21, b22;
    frame_apply_t(f, cj.v[1], cj.v[2], m11, m12);
    frame_apply_t(f, cj.v[3], cj.v[4], m21, m22);
    frame_apply_t(f0, m11, m21, b11, b21);
    frame_apply_t(f0, m12, m22, b12, b22);
    g0 = fma(cj.v[0], a0, g0);
    g1 = fma(b11, a1, fma(b21, a2, g1));
    g2 = fma(b12, a1, fma(b22, a2, g2));
  }
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) {
    g0 += __shfl_xor(g0, off, 16);
    g1 += __shfl_xor(g1, off, 16);
    g2 += __shfl_xor(g2, off, 16);
  }
  if (lane == 0) {
    const int c = gt_cell[row];
    const size_t nn = (size_t)6 * n * n;
    gq[c] += g0;
    gq[nn + c] += g1;
    gq[2 * nn + c] += g2;
  }
}

// ---------------------------------------------------------------------------
// Launcher of the whole adjoint
// ---------------------------------------------------------------------------
template <int K, bool W, int M, bool TP>
static int vjp_t(const VjpArgs& a, int step, void* stream) {
  const hipStream_t s = (hipStream_t)stream;
  const GridScalars& gs = a.gs;
  const int n = gs.n, P = gs.P;
  const int cells = 6 * n * n;
  switch (step) {
    case kVjpTraces:
      hipLaunchKernelGGL((k_vjp_traces<K, W, M, TP>), dim3((3 * cells + 63) / 64), dim3(64), 0, s, a.tab, gs, a.q, a.T,
                         a.topo);
      break;
    case kVjpPoints:
      hipLaunchKernelGGL((k_vjp_points<K, W, M, TP>), dim3((12 * n * (n + 1) + cells + 63) / 64), dim3(64), 0, s,
                         a.tab, a.itab, gs, a.T, a.w, a.Lam, a.topo, a.Lder);
      break;
    case kVjpEdges: {
      const int ept = 24 * n * M;
      hipLaunchKernelGGL((k_vjp_edges<K, W, M, TP>), dim3((ept + 63) / 64), dim3(64), 0, s, a.tab, a.itab, gs, a.T,
                         a.w, a.Lam, a.topo);
      break;
    }
    case kVjpWeno:
      if constexpr (W)
        hipLaunchKernelGGL((k_vjp_weno<K, W, M, TP>), dim3((a.nv * cells + 63) / 64), dim3(64), 0, s, a.tab, gs, a.q,
                           a.Lam, a.Dl, a.topo, a.Lder, a.v0, a.nv);
      else
        hipLaunchKernelGGL((k_vjp_tpp<K, W, M, TP>), dim3((a.nv * cells + 63) / 64), dim3(64), 0, s, a.tab, gs,
                           a.Lam, a.Dl, a.Lder, a.v0, a.nv);
      break;
    case kVjpGather: {
      const size_t padded = (size_t)a.nv * 6 * P * P;
      hipLaunchKernelGGL((k_vjp_gather<K, W, M>), dim3((unsigned)((padded + 255) / 256)), dim3(256), 0, s, a.tab, gs,
                         a.Lam, a.Dl, a.gpad, a.v0, a.nv);
      break;
    }
    case kVjpGhostT:
      hipLaunchKernelGGL(k_vjp_interior, dim3((cells + 255) / 256), dim3(256), 0, s, n, P, gs.r, a.gpad, a.gq);
      if (a.gt_blocks > 0)
        hipLaunchKernelGGL(k_vjp_ghost_t_lds, dim3((unsigned)((a.gt_blocks + kXcds - 1) / kXcds * kXcds)),
                           dim3(256), (size_t)3 * a.gt_umax * sizeof(double), s, a.gt_blocks, a.gt_border,
                           a.gt_rows, n, P, a.gt_umax, a.gt_cell, a.gt_ptr, a.gt_bptr, a.gt_bsrc, a.gt_lidx,
                           a.gt_ref, a.gcval, a.gpad, a.gq);
      else if (a.gt_rows > 0)
        hipLaunchKernelGGL(k_vjp_ghost_t, dim3((unsigned)(((size_t)a.gt_rows * 16 + 255) / 256)), dim3(256), 0, s,
                           a.gt_rows, n, P, a.gt_cell, a.gt_ptr, a.gt_row, a.gt_ref, a.gcval, a.gpad, a.gq);
      break;
    default:
      return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

template <bool TP>
static int launch_vjp_t(int k, int weno, const VjpArgs& a, int step, void* stream) {
  if (!weno) {
    switch (k) {
      case 3: return vjp_t<3, false, 2, TP>(a, step, stream);
      case 5: return vjp_t<5, false, 3, TP>(a, step, stream);
      case 7: return vjp_t<7, false, 4, TP>(a, step, stream);
      case 9: return vjp_t<9, false, 5, TP>(a, step, stream);
      case 11: return vjp_t<11, false, 6, TP>(a, step, stream);
      case 13: return vjp_t<13, false, 7, TP>(a, step, stream);
    }
  } else {
    switch (k) {
      case 3: return vjp_t<3, true, 2, TP>(a, step, stream);
      case 5: return vjp_t<5, true, 3, TP>(a, step, stream);
    }
  }
  return (int)hipErrorInvalidValue;
}

int launch_vjp(int k, int weno, const VjpArgs& a, int step, void* stream) {
  return a.topo.sbar ? launch_vjp_t<true>(k, weno, a, step, stream) : launch_vjp_t<false>(k, weno, a, step, stream);
}

}  // namespace hope
