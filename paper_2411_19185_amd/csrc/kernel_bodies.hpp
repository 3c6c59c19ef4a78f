// Device bodies of the HOPE right-hand-side kernels, shared by the kernels of
// one grid (kernels.hip) and the batched ensemble kernels (batch.hip).
//
//  halo_row    one row of the ghost fill g = G q (appendix (7.12)), from the
//              state or from a workgroup's LDS copy of the cells its rows read
//  edge_trace  at one panel-edge side, the neighbour panel's own trace,
//              converted into this panel's variables (3.26)-(3.29)
//  stage_tile  one work item of the fused stage: reconstruction (TPP (3.14)
//              or genuine 2D WENO (3.16)-(3.25)), LMARS (3.30)-(3.38), Gauss
//              quadrature (3.5)-(3.6) with sources (2.2)-(2.3), the tendency
//              (3.1) and an optional Runge-Kutta combination
//
// stage_tile marches: a workgroup of three wavefronts owns a strip of up to 62
// interior columns of one panel (lanes 1..62; lanes 0 and 63 are the strip's
// ring columns), or two strips of up to 30 (one per half of the lanes), and a
// segment of rows, walking up the rows.  The 2r+1 stencil rows of the strip
// sit in an LDS ring buffer (one new row per step, fetched a step ahead).  At
// each row wavefront v reconstructs variable v of every lane's cell into LDS;
// then wavefront 0 evaluates the flux through each lane's left edge (left
// state: lane L-1's right trace), wavefront 1 the flux through the bottom edge
// (left state: the top traces of the row below, carried from the previous
// step) and wavefront 2 the sources.  The only traces that go to HBM are those
// of the rows beside a segment boundary, for the segment seams.
//
// The grid's constant tables are one buffer read through the constant address
// space: with uniform addresses those reads are scalar loads into SGPRs.
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace hope {

// Frame codes of the rotation-compressed ghost map (GhostDev).  A row of a
// canonical momentum block, (c1, c2), acts on the canonical frame of the
// cell read; acting instead on that cell's own frame it is T (c1, c2), T the
// code's matrix.  A canonical ghost momentum (c1, c2) in the ghost's panel
// frame is also T (c1, c2).  Signed permutations: exact.
__device__ __forceinline__ void frame_apply(int f, double c1, double c2, double& g1, double& g2) {
  const bool sw = f & 1;
  const double sx = (f & 2) ? -1.0 : 1.0, sy = (f & 4) ? -1.0 : 1.0;
  g1 = sx * (sw ? c2 : c1);
  g2 = sy * (sw ? c1 : c2);
}

// one ghost row of g = G q, reduced over LANES lanes (lane = 0.. of the
// group): entries in column order, values from the row's canonical row;
// src(k, ce, a0, a1, a2) gives entry k's ce (canonical value and frame code)
// and the three variables of its cell (from the state, or from the LDS copy
// of the LDS-staged fill: the same values)
template <int LANES, typename Src>
__device__ __forceinline__ void halo_row_from(const GhostDev& g, double* __restrict__ q, size_t plane, int row,
                                              int lane, Src src) {
  const int b = g.ptr[row], e = g.ptr[row + 1];
  const int info = g.info[row];
  const GhostVal* cv = g.cval + (info & 0x0fffffff);
  double mass = 0, mu = 0, mv = 0;
  for (int k = b + lane; k < e; k += LANES) {
    int ce;
    double a0, a1, a2;
    src(k, ce, a0, a1, a2);
    const int j = ce & 0x1fff, f = ce >> 13;
    const GhostVal cj = cv[j];
    double w1, w2, w3, w4;
    frame_apply(f, cj.v[1], cj.v[2], w1, w2);
    frame_apply(f, cj.v[3], cj.v[4], w3, w4);
    mass = fma(cj.v[0], a0, mass);
    mu = fma(w1, a1, fma(w2, a2, mu));
    mv = fma(w3, a1, fma(w4, a2, mv));
  }
#pragma unroll
  for (int off = LANES / 2; off > 0; off >>= 1) {
    mass += __shfl_xor(mass, off, LANES);
    mu += __shfl_xor(mu, off, LANES);
    mv += __shfl_xor(mv, off, LANES);
  }
  if (lane == 0) {
    const int d = g.dst[row];
    double gu, gv;
    frame_apply(info >> 28, mu, mv, gu, gv);
    q[d] = mass;
    q[plane + d] = gu;
    q[2 * (size_t)plane + d] = gv;
  }
}

// one ghost row reading the state itself
template <int LANES>
__device__ __forceinline__ void halo_row(const GhostDev& g, double* __restrict__ q, size_t plane, int row, int lane) {
  const double* q1 = q + plane;
  const double* q2 = q + 2 * (size_t)plane;
  halo_row_from<LANES>(g, q, plane, row, lane, [&](int k, int& ce, double& a0, double& a1, double& a2) {
    const GhostEnt en = g.ent[k];
    const int c = en.col;
    ce = en.ce;
    a0 = q[c];
    a1 = q1[c];
    a2 = q2[c];
  });
}

// the converted neighbour trace at the panel-edge side idx (0 <= idx < 24 n),
// computed by a group of 4 consecutive lanes: lane g of the group
// reconstructs variable min(g, 2) (lane 3 repeats variable 2, so the group
// takes no divergent path), the group exchanges its values, and lane g < 3
// writes component g of the converted trace (3.26)-(3.29)
// With topography (TP) the mass is reconstructed as sqrtG phi_t (the cell
// averages of sqrtG phi_s added to the stencil), and the converted trace is
// the layer's own sqrtG phi again: sqrtG phi_s at this panel's point removed.
constexpr int kEdgeLanes = 4;

template <int K, bool W, int M, bool TP = false>
__device__ __forceinline__ void edge_trace(cdp tab, cip itab, const GridScalars& gs, const double* __restrict__ q,
                                           double* __restrict__ bt, int idx, int g, const TopoDev& tp = TopoDev()) {
  using C = Cfg<K, W, M>;
  const int n = gs.n, P = gs.P;
  const TabOffsets O = tab_offsets(K, W, M, n);
  const size_t vs = (size_t)6 * P * P;
  const int v = min(g, 2);
  const double* c0 = q + itab[O.i_cell + idx] + v * vs;
  const double* s0 = TP ? tp.sbar + itab[O.i_cell + idx] : nullptr;
  const int sd = itab[O.i_side + idx];
  const int rev = itab[O.i_rev + idx];
  double vals[M];
  {
    auto at = [&](int dy, int dx) -> double {
      if constexpr (TP) return c0[dy * P + dx] + (v == 0 ? s0[dy * P + dx] : 0.0);
      else return c0[dy * P + dx];
    };
    double kap[W ? C::S : 1];
    if constexpr (W) weno_kappa<K, W, M>(tab, gs.eps, at, [&](int j, double x) { kap[j] = x; });
    auto kf = [&](int j) -> double { return kap[j]; };
    double xr[C::XR];
    if (sd < 2) {
      xpass<K, W, M>(tab, sd, at, xr);
      if constexpr (W) {
        WCol<K, M> col;
        wcol<K, W, M>(tab, sd, xr, kf, col);
#pragma unroll
        for (int h = 0; h < M; ++h) vals[h] = wpoint<K, W, M>(tab, sd, 2 + h, sd * M + h, col);
      } else {
#pragma unroll
        for (int h = 0; h < M; ++h) vals[h] = point<K, W, M>(tab, 2 + h, sd * M + h, xr, kf);
      }
    } else {
#pragma unroll
      for (int h = 0; h < M; ++h) {
        xpass<K, W, M>(tab, 2 + h, at, xr);
        if constexpr (W) {
          WCol<K, M> col;
          wcol<K, W, M>(tab, 2 + h, xr, kf, col);
          vals[h] = wpoint<K, W, M>(tab, 2 + h, sd - 2, (sd == 2 ? 2 * M : 3 * M) + h, col);
        } else {
          vals[h] = point<K, W, M>(tab, sd - 2, (sd == 2 ? 2 * M : 3 * M) + h, xr, kf);
        }
      }
    }
  }
#pragma unroll
  for (int h = 0; h < M; ++h) {
    const double mine = rev ? vals[M - 1 - h] : vals[h];
    const double a0 = __shfl(mine, 0, kEdgeLanes), a1 = __shfl(mine, 1, kEdgeLanes), a2 = __shfl(mine, 2, kEdgeLanes);
    cdp cv = tab + O.bt_conv + ((size_t)idx * M + h) * 5;
    double* o = bt + ((size_t)idx * M + h) * 3;
    if constexpr (TP) {
      if (g == 0) o[0] = cv[0] * a0 - topo_side_point<M>(tp, n, idx, h);
    } else {
      if (g == 0) o[0] = cv[0] * a0;
    }
    if (g == 1) o[1] = cv[1] * a1 + cv[2] * a2;
    if (g == 2) o[2] = cv[3] * a1 + cv[4] * a2;
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
  int half;                 // strips of <= kHalfStrip columns: two per workgroup, 32 lanes each
  TopoDev tp;               // bottom topography tables (used by the TP kernels only)
  double* seam = nullptr;   // segment seams (SeamLayout), or null: segments re-reconstruct their neighbours' rows
};



// Segment seams (SeamLayout) at WENO5 and TPP9 and up, in the single-grid and
// batched stages alike: at the cheaper orders the seam kernel and its stores
// cost more than the boundary rows they save.
template <int K, bool W, int M>
constexpr bool kSeams = (W && K == 5) || K >= 9;

// The fused stage runs three wavefronts per work item: in the reconstruction
// phase wavefront v reconstructs variable v, so that each keeps only one
// variable's stencil passes and WENO weights live; the flux, source and
// assembly phases are then split between the three.
constexpr int kStageThreads = 192;

// with topography, the cell average of psi_B (2.14) of every lane's cell in
// the current row, formed by wavefront 0 (the mass) for wavefront 2 (sources)
template <bool TP>
struct TopoSmem {};
template <>
struct TopoSmem<true> {
  double psb[2][64];
};

template <int K, bool W, int M, bool TP = false>
struct StageSmem : TopoSmem<TP> {
  // window columns: one strip of up to 64 lanes plus 2R, or two half strips
  // of 32 lanes plus 2R each
  static constexpr int R = (K - 1) / 2, NR = 2 * R + 1, CW = 64 + 4 * R;
  // TPP orders 11 and 13 take the cell nodes in chunks of HC node columns
  // (the sources of a chunk are added before the next chunk is
  // reconstructed), so that two workgroups fit in a CU's LDS instead of one;
  // the lower orders keep all M x M, which measured faster for them.
  static constexpr bool kChunk = !W && K >= 11;
  static constexpr int HC = kChunk ? (K >= 13 ? 1 : 2) : M;
  static constexpr int NCH = (M + HC - 1) / HC;
  // slots of pts: left edge, right edge, bottom edge (M each), then the cell
  // nodes of one chunk (M x HC); a row's top traces stay in the registers of
  // the wavefront that computed them until they move to ptop
  static constexpr int PL = 0, PR = M, PB = 2 * M, PI = 3 * M, NP = 3 * M + M * HC;
  double sq[3][NR][CW];     // stencil window: NR padded rows (column c of a strip's part = padded column i0-1+c)
  double pts[3][NP][64];    // the current row's values at the points of every lane's cell
  double ptop[3][M][64];    // top traces of the row below
};

// one work item (panel, strip, segment) of the fused stage; fcb = the 6 x 3
// Coriolis coefficients of the grid (or of one ensemble member).  Called by
// all kStageThreads threads of the workgroup.
//
// The strip's lanes: lane L works on column i0-1+L; lanes 1..strip_w own the
// strip's cells, lanes 0 and strip_w+1 are its ring columns.  Walking up the
// rows j0..j1 of the segment, each step j (j < j1) reconstructs row j,
// evaluates the flux through every lane's left and bottom edge and the
// sources, finishes row j-1 (whose top flux is row j's bottom flux) and forms
// row j's partial tendency.  Step j1 only supplies the top flux of row j1-1.
//
// With bottom topography (TP, (2.13)-(2.14)) the window holds sqrtG phi_t for
// the mass (q + the cell averages of sqrtG phi_s); wavefront 0 subtracts
// sqrtG phi_s from each of its point values, so every later phase sees the
// layer's own sqrtG phi, and forms psi_B of the row from the derivative of
// the centred order-k polynomial of sqrtG phi_t at the cell nodes; the LMARS
// pressure adds phi_s.
template <int K, bool W, int M, bool TP = false, bool SEAMS = false>
__device__ __forceinline__ void stage_tile(const double* __restrict__ tab_, cdp fcb, const GridScalars& gs,
                                           const StageArgs& A, int item, StageSmem<K, W, M, TP>& sm) {
  using C = Cfg<K, W, M>;
  constexpr int R = C::R, S = C::S, NR = C::NR, XR = C::XR;
  constexpr int CW = StageSmem<K, W, M>::CW;       // window columns allocated
  constexpr int HW = 32 + 2 * R;                   // window columns of a half strip
  cdp tab = (cdp)tab_;
  const int n = gs.n, P = gs.P;
  const TabOffsets O = tab_offsets(K, W, M, n);
  const size_t plane = (size_t)P * P;
  const size_t vs = 6 * plane;
  const bool half = A.half != 0;
  const int seg = item % A.n_segs;
  const int colpos = item / A.n_segs;              // strip column, or pair of strip columns
  const int ncols = 6 * A.n_strips;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // this wavefront's variable / role
  const int grp = half ? lane >> 5 : 0;            // which half strip (0 in full mode)
  const int gl = half ? lane & 31 : lane;          // lane within the strip
  // strip column of half g (clamped; the second half of the last pair may be empty)
  auto col_of = [&](int g) { return min(half ? 2 * colpos + g : colpos, ncols - 1); };
  const bool live = !half || 2 * colpos + grp < ncols;
  const int scol = col_of(grp);
  const int strip = scol % A.n_strips;
  const int p = scol / A.n_strips;
  const int i0 = strip * A.strip_w;
  const int i1 = live ? min(n, i0 + A.strip_w) : i0;   // owned columns [i0, i1)
  const int i = i0 - 1 + gl;                       // this lane's column
  const bool in_strip = live && (i >= i0 - 1) && (i <= i1);
  const bool real = in_strip && i >= 0 && i < n;   // a cell this lane can reconstruct
  const bool owner = i >= i0 && i < i1;            // a cell whose result this lane writes
  const int wc = (half ? grp * HW : 0) + gl + R;   // window column of this lane's cell
  const int j0 = seg * A.seg_h;
  const int j1 = min(n, j0 + A.seg_h);
  const double invd = gs.inv_delta;
  const double ia = 1.0 / gs.radius;
  const double* btp = A.bt + (size_t)p * 4 * n * M * 3;
  const int ic = max(0, min(n - 1, i));            // clamped column for table reads
  cdp Xg = tab + O.Xg, sqg = tab + O.sqg, Xe = tab + O.Xe, sqe = tab + O.sqe, gw = tab + C::O.gw;

  // ---- window rows (all threads) -------------------------------------------
  constexpr int PER = (3 * CW + kStageThreads - 1) / kStageThreads;
  auto fetch = [&](int pr, double* buf) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = tid + kStageThreads * k;
      const int v = idx / CW, c = idx % CW;
      const int g = half ? c / HW : 0, cc = half ? c % HW : c;
      const int sc = col_of(g);
      const int gc = (sc % A.n_strips) * A.strip_w - 1 + cc;
      const bool used = half ? g < 2 : c < 64 + 2 * R;
      const bool ok = idx < 3 * CW && used && pr >= 0 && pr < P && gc >= 0 && gc < P;
      const size_t off = (sc / A.n_strips) * plane + (size_t)pr * P + gc;
      if constexpr (TP) buf[k] = ok ? A.q[off + v * vs] + (v == 0 ? A.tp.sbar[off] : 0.0) : 0.0;
      else buf[k] = ok ? A.q[off + v * vs] : 0.0;
    }
  };
  auto store = [&](int pr, const double* buf) {
    const int slot = pr % NR;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = tid + kStageThreads * k;
      if (idx < 3 * CW) sm.sq[idx / CW][slot][idx % CW] = buf[k];
    }
  };
  // stencil of this wavefront's variable at offset (dy, dx) of the lane's cell in interior row pc
  auto win = [&](int pc) {
    return [&, pc](int dy, int dx) -> double { return sm.sq[wv][(pc + R + dy) % NR][wc + dx]; };
  };
  // WENO weights kappa_j of this wavefront's variable in row pc
  auto kappa = [&](int pc, double* kap) {
    if constexpr (W) weno_kappa<K, W, M>(tab, gs.eps, win(pc), [&](int j, double x) { kap[j] = x; });
  };
  auto pt = [&](int v, int k) -> double& { return sm.pts[v][k][lane]; };
  using SM = StageSmem<K, W, M>;
  // results of the flux phase, each written over a point slot that only its
  // writer read: the x flux through lane L's left edge over the left trace
  // (wavefront 0), the y flux over the bottom trace (wavefront 1) and the two
  // momentum sources over the first cell node of variables 0 and 1
  // (wavefront 2)
  auto fx = [&](int v, int l) -> double& { return sm.pts[v][SM::PL][l]; };
  auto fy = [&](int v) -> double& { return sm.pts[v][SM::PB][lane]; };
  auto src = [&](int c) -> double& { return sm.pts[c][SM::PI][lane]; };
  // topography: sqrtG phi_s at this lane's points of row pc (edge indices clamped
  // for the ring lanes, whose values at a panel edge are not used)
  const int ie_l = max(0, min(n, i)), ie_r = max(0, min(n, i + 1));
  auto s_xe = [&](int pc, int ie, int h) -> double {
    return A.tp.sx[(((size_t)p * n + pc) * (n + 1) + ie) * M + h];
  };
  auto s_ye = [&](int je, int h) -> double { return A.tp.sy[(((size_t)p * (n + 1) + je) * n + ic) * M + h]; };
  auto s_cq = [&](int pc, int w, int h) -> double {
    return A.tp.sc[((((size_t)p * n + pc) * n + ic) * M + w) * M + h];
  };
  // the layer's own mass at a point of this wavefront's variable: with
  // topography, wavefront 0 removes sqrtG phi_s from sqrtG phi_t
  auto layer = [&](double val, auto s_of) -> double {
    if constexpr (TP) return wv == 0 ? val - s_of() : val;
    else return val;
  };

  // ---- topography: psi_B of the row, by wavefront 0 --------------------------
  // centred (xc) and derivative (xd) x-passes of sqrtG phi_t at x axis point px
  auto tpass = [&](int pc, int px, double* xc, double* xd) {
    cdp wcc = tab + C::O.wc, wdd = tab + C::O.wd;
    auto at = win(pc);
#pragma unroll
    for (int row = 0; row < NR; ++row) {
      double a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int a = 0; a < K; ++a) {
        const double x = at(row - R, a - R);
        a0 = fma(wcc[px * K + a], x, a0);
        a1 = fma(wdd[px * K + a], x, a1);
      }
      xc[row] = a0;
      xd[row] = a1;
    }
  };
  // derivative x-pass only (TPP: the centred x-pass is the reconstruction's own)
  auto dpass = [&](int pc, int px, double* xd) {
    cdp wdd = tab + C::O.wd;
    auto at = win(pc);
#pragma unroll
    for (int row = 0; row < NR; ++row) {
      double a1 = 0.0;
#pragma unroll
      for (int a = 0; a < K; ++a) a1 = fma(wdd[px * K + a], at(row - R, a - R), a1);
      xd[row] = a1;
    }
  };
  // adds psi_B at the cell node (x node h, y node w) of row pc, where the
  // reconstructed sqrtG phi_t is T, weighted by the cell quadrature (3.6)
  auto psi_add = [&](int pc, int h, int w, double T, const double* xc, const double* xd, double& b1, double& b2) {
    cdp wcc = tab + C::O.wc, wdd = tab + C::O.wd;
    double Txi = 0.0, Teta = 0.0;
#pragma unroll
    for (int b = 0; b < K; ++b) {
      Txi = fma(wcc[(2 + w) * K + b], xd[b], Txi);
      Teta = fma(wdd[(2 + w) * K + b], xc[b], Teta);
    }
    double c1, c2;
    psi_b(T, Txi, Teta, Xg[ic * M + h], Xg[pc * M + w], s_cq(pc, w, h), invd, ia, c1, c2);
    const double g2 = gw[h] * gw[w];
    b1 = fma(g2, c1, b1);
    b2 = fma(g2, c2, b2);
  };

  // segment seams below row j0 (sb) and above row j1-1 (sa); SEAMS compiles
  // them in (the batched kernel runs without)
  const bool sb = SEAMS && A.seam && j0 > 0, sa = SEAMS && A.seam && j1 < n;
  // (32-bit offsets: a seam buffer holds at most 6 n^2 (6m + 11) / 2 elements)
  const int seam_ns = A.seam ? 6 * (A.n_segs - 1) * n : 0;
  auto seam_at = [&](int u, int f) -> double& { return A.seam[f * seam_ns + (p * (A.n_segs - 1) + (u - 1)) * n + i]; };
  // the traces a seam takes: the bottom traces of row j0 (seam below) and the
  // top traces of row j1-1 (seam above).  TPP stores them as the row's
  // reconstruction forms them; WENO, whose unrolled reconstruction holds more
  // registers, from LDS afterwards (the bottom traces from the point slots at
  // the end of step j0, the top traces from ptop after the loop), which
  // measured faster for WENO and slower for TPP
  auto seam_traces = [&](int pc, int h, double bot, double topv) {
    if constexpr (!W) {
      if (sb && pc == j0 && owner) seam_at(seg, SeamLayout::tb(M, h, wv)) = bot;
      if (sa && pc == j1 - 1 && owner) seam_at(seg + 1, SeamLayout::tt(M, h, wv)) = topv;
    }
  };
  // ---- reconstruction phase: wavefront wv, variable wv ----------------------
  // every point of row pc
  auto recon_row = [&](int pc, double* top) {
    double kap[W ? S : 1];
    kappa(pc, kap);
    auto kf = [&](int j) -> double { return kap[j]; };
    double xr[XR];
    double pb1 = 0.0, pb2 = 0.0;          // topography: psi_B of the row (wavefront 0)
    if constexpr (W) {
      // WENO by columns: the sums over sub-stencil columns are shared by the
      // points of one x axis point
      WCol<K, M> col;
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        asm volatile("" ::: "memory");
        xpass<K, W, M>(tab, sd, win(pc), xr);
        wcol<K, W, M>(tab, sd, xr, kf, col);
#pragma unroll
        for (int h = 0; h < M; ++h)
          pt(wv, sd * M + h) = layer(wpoint<K, W, M>(tab, sd, 2 + h, sd * M + h, col),
                                     [&] { return s_xe(pc, sd ? ie_r : ie_l, h); });
      }
#pragma unroll
      for (int h = 0; h < M; ++h) {
        asm volatile("" ::: "memory");
        xpass<K, W, M>(tab, 2 + h, win(pc), xr);
        wcol<K, W, M>(tab, 2 + h, xr, kf, col);
        const double vb = layer(wpoint<K, W, M>(tab, 2 + h, 0, 2 * M + h, col), [&] { return s_ye(pc, h); });
        const double vt = layer(wpoint<K, W, M>(tab, 2 + h, 1, 3 * M + h, col), [&] { return s_ye(pc + 1, h); });
        pt(wv, SM::PB + h) = vb;
        top[h] = vt;
        seam_traces(pc, h, vb, vt);
        if constexpr (TP) {
          double xc[NR], xd[NR];
          if (wv == 0) tpass(pc, 2 + h, xc, xd);
#pragma unroll
          for (int w = 0; w < M; ++w) {
            const double v = wpoint<K, W, M>(tab, 2 + h, 2 + w, 4 * M + w * M + h, col);
            if (wv == 0) psi_add(pc, h, w, v, xc, xd, pb1, pb2);
            pt(wv, SM::PI + w * M + h) = layer(v, [&] { return s_cq(pc, w, h); });
          }
        } else {
#pragma unroll
          for (int w = 0; w < M; ++w)
            pt(wv, SM::PI + w * M + h) = wpoint<K, W, M>(tab, 2 + h, 2 + w, 4 * M + w * M + h, col);
        }
      }
    } else {
      asm volatile("" ::: "memory");
      xpass<K, W, M>(tab, 0, win(pc), xr);
#pragma unroll
      for (int h = 0; h < M; ++h) pt(wv, h) = layer(point<K, W, M>(tab, 2 + h, h, xr, kf), [&] { return s_xe(pc, ie_l, h); });
      asm volatile("" ::: "memory");
      xpass<K, W, M>(tab, 1, win(pc), xr);
#pragma unroll
      for (int h = 0; h < M; ++h)
        pt(wv, M + h) = layer(point<K, W, M>(tab, 2 + h, M + h, xr, kf), [&] { return s_xe(pc, ie_r, h); });
#pragma unroll 1
      for (int h = 0; h < M; ++h) {
        asm volatile("" ::: "memory");
        xpass<K, W, M>(tab, 2 + h, win(pc), xr);
        const double vb = layer(point<K, W, M>(tab, 0, 2 * M + h, xr, kf), [&] { return s_ye(pc, h); });
        const double vt = layer(point<K, W, M>(tab, 1, 3 * M + h, xr, kf), [&] { return s_ye(pc + 1, h); });
        pt(wv, SM::PB + h) = vb;
        top[h] = vt;
        seam_traces(pc, h, vb, vt);
        if constexpr (TP) {
          double xd[NR];
          if (wv == 0) dpass(pc, 2 + h, xd);
#pragma unroll
          for (int w = 0; w < M; ++w) {
            const double v = point<K, W, M>(tab, 2 + w, 4 * M + w * M + h, xr, kf);
            if (wv == 0) psi_add(pc, h, w, v, xr, xd, pb1, pb2);
            pt(wv, SM::PI + w * M + h) = layer(v, [&] { return s_cq(pc, w, h); });
          }
        } else {
#pragma unroll
          for (int w = 0; w < M; ++w)
            pt(wv, SM::PI + w * M + h) = point<K, W, M>(tab, 2 + w, 4 * M + w * M + h, xr, kf);
        }
      }
    }
    if constexpr (TP) {
      if (wv == 0) {
        sm.psb[0][lane] = pb1;
        sm.psb[1][lane] = pb2;
      }
    }
  };
  // top (side 1) or bottom (side 0) traces of row pc, into dst(h)
  auto recon_side = [&](int pc, int side, auto dst) {
    double kap[W ? S : 1];
    kappa(pc, kap);
    auto kf = [&](int j) -> double { return kap[j]; };
#pragma unroll 1
    for (int h = 0; h < M; ++h) {
      double xr[XR];
      asm volatile("" ::: "memory");
      xpass<K, W, M>(tab, 2 + h, win(pc), xr);
      if constexpr (W) {
        // the same arithmetic as recon_row, so that a trace does not depend on
        // whether its row is reconstructed whole or only for its side
        WCol<K, M> col;
        wcol<K, W, M>(tab, 2 + h, xr, kf, col);
        dst(h) = layer(wpoint<K, W, M>(tab, 2 + h, side, (2 + side) * M + h, col),
                       [&] { return s_ye(pc + side, h); });
      } else {
        dst(h) = layer(point<K, W, M>(tab, side, (2 + side) * M + h, xr, kf), [&] { return s_ye(pc + side, h); });
      }
    }
  };

  // ---- flux phase ------------------------------------------------------------
  // wavefront 1: flux through the bottom edge of row j (qL: top trace of row
  // j-1 in ptop, qR: bottom trace of row j in pts)
  auto yflux = [&](int j) {
    double gb[3] = {0.0, 0.0, 0.0};
    // the lane's Gauss-node tables, requested one node ahead
    double xg_n = Xg[ic * M], sq_n = sqg[ic * M];
#pragma unroll 1
    for (int h = 0; h < M; ++h) {
      const double xg = xg_n, sqv = sq_n;
      if (h + 1 < M) {
        xg_n = Xg[ic * M + h + 1];
        sq_n = sqg[ic * M + h + 1];
      }
      double qL[3], qR[3];
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        const double dflt = v == 0 ? 1.0 : 0.0;
        qL[v] = real ? sm.ptop[v][h][lane] : dflt;
        qR[v] = real ? pt(v, SM::PB + h) : dflt;
      }
      double F[3];
      lmars<TP>(qL, qR, xg, Xe[j], sqv, sqe[j], 1, ia, F, TP ? s_ye(j, h) : 0.0);
#pragma unroll
      for (int v = 0; v < 3; ++v) gb[v] = fma(gw[h], F[v], gb[v]);
    }
#pragma unroll
    for (int v = 0; v < 3; ++v) fy(v) = gb[v];
  };
  // wavefront 0: flux through the left edge of each lane's column in row j;
  // panel edges take the neighbour's converted trace
  auto xflux = [&](int j) {
    const int ie = max(0, min(n, i));
    const double Xei = tab[O.Xe + ie], sqxe = tab[O.sqe + ie];
    const bool xdead = !(in_strip && i >= 0 && i <= n && gl >= 1);
    const int ll = max(lane - 1, 0);
    double fl[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
    for (int h = 0; h < M; ++h) {
      double qL[3], qR[3];
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        const double dflt = v == 0 ? 1.0 : 0.0;
        const double l = sm.pts[v][SM::PR + h][ll];
        const double r = pt(v, SM::PL + h);
        // only the lanes on a panel edge read the neighbour's trace
        qL[v] = xdead ? dflt : (i == 0 ? btp[(((size_t)0 * n + j) * M + h) * 3 + v] : l);
        qR[v] = xdead ? dflt : (i == n ? btp[(((size_t)1 * n + j) * M + h) * 3 + v] : r);
      }
      double F[3];
      lmars<TP>(qL, qR, Xei, Xg[j * M + h], sqxe, sqg[j * M + h], 0, ia, F, TP ? s_xe(j, ie, h) : 0.0);
#pragma unroll
      for (int v = 0; v < 3; ++v) fl[v] = fma(gw[h], F[v], fl[v]);
    }
#pragma unroll
    for (int v = 0; v < 3; ++v) fx(v, lane) = fl[v];
  };
  // wavefront 2: sources of the node columns [h0, h1) of row j, whose values
  // are in the chunk slots (chunked mode), accumulated into s1, s2 in the
  // order of sources_row
  auto sources_chunk = [&](int j, int h0, int h1, double& s1, double& s2) {
    cdp fc = fcb + p * 3;
    const double Lx0 = fc[0], LxX = fc[1], LxY = fc[2];
#pragma unroll 1
    for (int h = h0; h < h1; ++h) {
      const double X = Xg[ic * M + h];
#pragma unroll
      for (int w = 0; w < M; ++w) {
        double cq[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) cq[v] = real ? pt(v, SM::PI + w * SM::HC + (h - h0)) : (v == 0 ? 1.0 : 0.0);
        const double Y = Xg[j * M + w];
        double a1, a2;
        sources(cq[0], cq[1], cq[2], X, Y, Lx0 + LxX * X + LxY * Y, gs.omega2, a1, a2);
        const double g2 = gw[h] * gw[w];
        s1 = fma(g2, a1, s1);
        s2 = fma(g2, a2, s2);
      }
    }
  };
  // chunked TPP: every point of row pc, the cell nodes chunk by chunk, with
  // wavefront 2 adding each chunk's sources between two barriers (all
  // threads pass the same barriers)
  auto recon_row_chunked = [&](int pc, double* top, double& s1, double& s2) {
    double kap[1];
    auto kf = [&](int jj) -> double { return kap[jj]; };
    double xr[XR];
    double pb1 = 0.0, pb2 = 0.0;          // topography: psi_B of the row (wavefront 0)
    asm volatile("" ::: "memory");
    xpass<K, W, M>(tab, 0, win(pc), xr);
#pragma unroll
    for (int h = 0; h < M; ++h) pt(wv, h) = layer(point<K, W, M>(tab, 2 + h, h, xr, kf), [&] { return s_xe(pc, ie_l, h); });
    asm volatile("" ::: "memory");
    xpass<K, W, M>(tab, 1, win(pc), xr);
#pragma unroll
    for (int h = 0; h < M; ++h)
      pt(wv, M + h) = layer(point<K, W, M>(tab, 2 + h, M + h, xr, kf), [&] { return s_xe(pc, ie_r, h); });
    s1 = 0.0;
    s2 = 0.0;
#pragma unroll 1
    for (int c = 0; c < SM::NCH; ++c) {
      const int h0 = c * SM::HC, h1 = min(M, h0 + SM::HC);
#pragma unroll 1
      for (int h = h0; h < h1; ++h) {
        asm volatile("" ::: "memory");
        xpass<K, W, M>(tab, 2 + h, win(pc), xr);
        const double vb = layer(point<K, W, M>(tab, 0, 2 * M + h, xr, kf), [&] { return s_ye(pc, h); });
        const double vt = layer(point<K, W, M>(tab, 1, 3 * M + h, xr, kf), [&] { return s_ye(pc + 1, h); });
        pt(wv, SM::PB + h) = vb;
        top[h] = vt;
        seam_traces(pc, h, vb, vt);
        if constexpr (TP) {
          double xd[NR];
          if (wv == 0) dpass(pc, 2 + h, xd);
#pragma unroll
          for (int w = 0; w < M; ++w) {
            const double v = point<K, W, M>(tab, 2 + w, 4 * M + w * M + h, xr, kf);
            if (wv == 0) psi_add(pc, h, w, v, xr, xd, pb1, pb2);
            pt(wv, SM::PI + w * SM::HC + (h - h0)) = layer(v, [&] { return s_cq(pc, w, h); });
          }
        } else {
#pragma unroll
          for (int w = 0; w < M; ++w)
            pt(wv, SM::PI + w * SM::HC + (h - h0)) = point<K, W, M>(tab, 2 + w, 4 * M + w * M + h, xr, kf);
        }
      }
      __syncthreads();
      if (wv == 2) sources_chunk(pc, h0, h1, s1, s2);
      if (c + 1 < SM::NCH) __syncthreads();
    }
    if constexpr (TP) {
      if (wv == 0) {
        sm.psb[0][lane] = pb1;
        sm.psb[1][lane] = pb2;
      }
    }
  };
  // wavefront 2: metric and Coriolis sources of row j (cell quadrature)
  auto sources_row = [&](int j) {
    cdp fc = fcb + p * 3;
    const double Lx0 = fc[0], LxX = fc[1], LxY = fc[2];
    double s1 = 0.0, s2 = 0.0;
    double x_n = Xg[ic * M];
#pragma unroll 1
    for (int h = 0; h < M; ++h) {
      const double X = x_n;
      if (h + 1 < M) x_n = Xg[ic * M + h + 1];
#pragma unroll
      for (int w = 0; w < M; ++w) {
        double cq[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) cq[v] = real ? pt(v, SM::PI + w * M + h) : (v == 0 ? 1.0 : 0.0);
        const double Y = Xg[j * M + w];
        double a1, a2;
        sources(cq[0], cq[1], cq[2], X, Y, Lx0 + LxX * X + LxY * Y, gs.omega2, a1, a2);
        const double g2 = gw[h] * gw[w];
        s1 = fma(g2, a1, s1);
        s2 = fma(g2, a2, s2);
      }
    }
    if constexpr (TP) {
      s1 += sm.psb[0][lane];
      s2 += sm.psb[1][lane];
    }
    src(0) = s1;
    src(1) = s2;
  };

  // ---- prologue: window and the top traces of row j0-1 ------------------
  double nxt[PER];
  for (int pr = sb ? j0 : max(0, j0 - 1); pr < j0 + 2 * R; ++pr) {
    fetch(pr, nxt);
    store(pr, nxt);
  }
  fetch(j0 + 2 * R, nxt);          // row needed by the first step
  __syncthreads();
  if (j0 == 0) {
#pragma unroll
    for (int h = 0; h < M; ++h)
      sm.ptop[wv][h][lane] = real ? btp[(((size_t)2 * n + ic) * M + h) * 3 + wv] : (wv ? 0.0 : 1.0);
  } else if (!sb) {
    recon_side(j0 - 1, 1, [&](int h) -> double& { return sm.ptop[wv][h][lane]; });
  }
  double acc = 0.0;                // this wavefront's variable: partial tendency of the previous row
  double top[M];                   // this wavefront's variable: top traces of the current row

  for (int j = j0; j <= j1; ++j) {
    const bool last = (j == j1);
    // the window of step j holds padded rows j .. j+2R; row j+2R was fetched
    // during the previous step and replaces row j-1, no longer read
    const bool have = !(last && (j1 == n || sa)) && (j + 2 * R) < P;
    // the slot of row j+2R held padded row j-1, last read by the previous
    // step's reconstruction (behind its flux barriers) or, in the first step,
    // by the prologue's top traces
    if (j == j0) __syncthreads();
    if (have) store(j + 2 * R, nxt);
    __syncthreads();
    const bool want = (j + 1 < j1 || (j + 1 == j1 && j1 < n && !sa)) && (j + 2 * R + 1) < P;
    if (want) fetch(j + 2 * R + 1, nxt);
    double s1c = 0.0, s2c = 0.0;     // chunked mode: this row's sources (wavefront 2)
    if (!last) {
      if constexpr (SM::kChunk) recon_row_chunked(j, top, s1c, s2c);
      else recon_row(j, top);
    } else if (j1 == n) {
      // bottom traces of the panel's top row: the neighbour's converted trace
#pragma unroll
      for (int h = 0; h < M; ++h) pt(wv, SM::PB + h) = real ? btp[(((size_t)3 * n + ic) * M + h) * 3 + wv] : 0.0;
    } else if (!sa) {
      recon_side(j, 0, [&](int h) -> double& { return pt(wv, SM::PB + h); });
    }
    __syncthreads();
    // the cell finished below: q^n is requested before the flux phase so that
    // its latency is hidden behind it; q_s is padded row jr+R of the window,
    // read before the next step's store may replace that row
    const bool fin = j > j0 && owner;
    const int jr = j - 1;
    const bool ex_lo = last && sa;                  // row j1-1 goes to the seam above
    const bool ex_gt = sb && j == j0 + 1;           // row j0's top flux goes to the seam below
    const bool wr = fin && !ex_lo && !ex_gt;        // the row is finished here
    const size_t o_in = wv * vs + p * plane + (size_t)(jr + R) * P + (i + R);
    const double qn_c = (wr && A.qn) ? A.qn[o_in] : 0.0;
    // (with topography the window's mass is sqrtG phi_t: q_s is read again)
    double qs_c = 0.0;
    if constexpr (TP) qs_c = wr ? (wv == 0 ? A.q[o_in] : sm.sq[wv][(jr + R) % NR][wc]) : 0.0;
    else qs_c = wr ? sm.sq[wv][(jr + R) % NR][wc] : 0.0;
    if (wv == 1 && !(last && sa) && !(j == j0 && sb)) yflux(j);
    if (!last) {
      if (wv == 0) xflux(j);
      if (wv == 2) {
        if constexpr (SM::kChunk) {
          if constexpr (TP) {
            s1c += sm.psb[0][lane];
            s2c += sm.psb[1][lane];
          }
          src(0) = s1c;
          src(1) = s2c;
        } else {
          sources_row(j);
        }
      }
    }
    __syncthreads();
    // ---- assembly: wavefront wv, variable wv -----------------------------
    const double gb = fy(wv);
    if (fin && ex_lo) {
      // row j1-1 goes to the seam above after the loop
    } else if (fin && ex_gt) {
      seam_at(seg, SeamLayout::hi_gt(M, wv)) = gb;
    } else if (fin) {
      // finish row j-1: its top flux is row j's bottom flux
      const double dq = fma(-gb, invd, acc);
      double val = A.cc * dq;
      if (A.cb != 0.0) val = fma(A.cb, qs_c, val);
      if (A.qn) val = fma(A.ca, qn_c, val);
      if (A.out_padded) {
        A.out[o_in] = val;
      } else {
        A.out[((size_t)(wv * 6 + p) * n + jr) * n + i] = val;
      }
    }
    if (last) break;
    const double fl = fx(wv, lane);
    const double fr = fx(wv, min(lane + 1, 63));
    if (j == j0 && sb) {
      // row j0: (WENO) its bottom traces, still in the point slots since the y
      // flux of this step was not formed, and the parts of its tendency other
      // than the bottom flux
      if (owner) {
        if constexpr (W) {
#pragma unroll
          for (int h = 0; h < M; ++h) seam_at(seg, SeamLayout::tb(M, h, wv)) = pt(wv, SM::PB + h);
        }
        seam_at(seg, SeamLayout::hi_x(M, wv)) = fl - fr;
        if (wv > 0) seam_at(seg, SeamLayout::hi_src(M, wv - 1)) = src(wv - 1);
      }
      acc = 0.0;
    } else {
      acc = wv == 0 ? (fl - fr + gb) * invd : fma(fl - fr + gb, invd, src(wv - 1));
    }
#pragma unroll
    for (int h = 0; h < M; ++h) sm.ptop[wv][h][lane] = top[h];
  }
  // row j1-1's partial tendency (all but its top flux) and (WENO) its top
  // traces, moved to ptop at the end of its step and left there by the last
  // step, for the seam above
  if (owner && sa) {
    seam_at(seg + 1, SeamLayout::lo_acc(M, wv)) = acc;
    if constexpr (W) {
#pragma unroll
      for (int h = 0; h < M; ++h) seam_at(seg + 1, SeamLayout::tt(M, h, wv)) = sm.ptop[wv][h][lane];
    }
  }
}

// One segment seam: the flux through the boundary e = u seg_h of panel p at
// column i (as the stage's y flux forms it), then the tendency (or Runge-Kutta
// combination) of rows e-1 and e, all three variables.  idx runs over
// 6 (n_segs-1) n records.
template <int K, bool W, int M, bool TP = false>
__device__ __forceinline__ void stage_seam(const double* __restrict__ tab_, const GridScalars& gs,
                                           const StageArgs& A, size_t idx) {
  using C = Cfg<K, W, M>;
  constexpr int R = C::R;
  cdp tab = (cdp)tab_;
  const int n = gs.n, P = gs.P;
  const TabOffsets O = tab_offsets(K, W, M, n);
  const size_t ns = (size_t)6 * (A.n_segs - 1) * n;
  const int i = (int)(idx % n);
  const int u = (int)((idx / n) % (A.n_segs - 1)) + 1;
  const int p = (int)(idx / ((size_t)(A.n_segs - 1) * n));
  const int e = u * A.seg_h;
  const double* rec = A.seam + idx;
  auto fld = [&](int f) -> double { return rec[(size_t)f * ns]; };
  const double invd = gs.inv_delta;
  const double ia = 1.0 / gs.radius;
  cdp Xg = tab + O.Xg, sqg = tab + O.sqg, Xe = tab + O.Xe, sqe = tab + O.sqe, gw = tab + C::O.gw;
  double gb[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
  for (int h = 0; h < M; ++h) {
    double qL[3], qR[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      qL[v] = fld(SeamLayout::tt(M, h, v));
      qR[v] = fld(SeamLayout::tb(M, h, v));
    }
    double F[3];
    const double sps = TP ? A.tp.sy[(((size_t)p * (n + 1) + e) * n + i) * M + h] : 0.0;
    lmars<TP>(qL, qR, Xg[i * M + h], Xe[e], sqg[i * M + h], sqe[e], 1, ia, F, sps);
#pragma unroll
    for (int v = 0; v < 3; ++v) gb[v] = fma(gw[h], F[v], gb[v]);
  }
  const size_t plane = (size_t)P * P, vs = 6 * plane;
  auto finish = [&](int v, int jr, double dq) {
    const size_t o_in = v * vs + p * plane + (size_t)(jr + R) * P + (i + R);
    double val = A.cc * dq;
    if (A.cb != 0.0) {
      // q_s as the stage reads it from its window (with topography the window
      // adds 0 to the momentum)
      double qs = A.q[o_in];
      if constexpr (TP) qs = v == 0 ? qs : qs + 0.0;
      val = fma(A.cb, qs, val);
    }
    if (A.qn) val = fma(A.ca, A.qn[o_in], val);
    if (A.out_padded) A.out[o_in] = val;
    else A.out[((size_t)(v * 6 + p) * n + jr) * n + i] = val;
  };
#pragma unroll
  for (int v = 0; v < 3; ++v) finish(v, e - 1, fma(-gb[v], invd, fld(SeamLayout::lo_acc(M, v))));
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const double x = fld(SeamLayout::hi_x(M, v));
    const double acc = v == 0 ? (x + gb[0]) * invd : fma(x + gb[v], invd, fld(SeamLayout::hi_src(M, v - 1)));
    finish(v, e, fma(-fld(SeamLayout::hi_gt(M, v)), invd, acc));
  }
}

}  // namespace hope
