// Host construction of every constant table of a HOPE grid: Gauss rules,
// reconstruction weights, WENO linear weights and smoothness forms, the
// equiangular metric tables, the exact ghost-cell map and the panel-edge
// trace maps.  Arithmetic is done in long double and rounded once to FP64.
#include <algorithm>
#include <array>
#include <cmath>
#include <limits>
#include <cstdio>
#include <cstring>

#include "hope.h"
#include "hope_internal.hpp"

namespace hope {
namespace {

using ld = long double;
const ld kPi = 3.141592653589793238462643383279502884L;

// ---------------------------------------------------------------------------
// Gauss-Legendre rule on [-1/2, 1/2], weights summing to one (eqs (3.5)-(3.6))
// ---------------------------------------------------------------------------
void gauss_rule(int m, std::vector<ld>& x, std::vector<ld>& w) {
  x.assign(m, 0);
  w.assign(m, 0);
  for (int i = 0; i < m; ++i) {
    ld z = std::cos(kPi * (i + 0.75L) / (m + 0.5L));  // Chebyshev-like start, descending
    ld dp = 0;
    for (int it = 0; it < 100; ++it) {
      ld p0 = 1, p1 = z;
      for (int k = 2; k <= m; ++k) {
        ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (m == 1) { p1 = z; p0 = 1; }
      dp = m * (z * p1 - p0) / (z * z - 1);
      ld dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-19L) break;
    }
    {
      ld p0 = 1, p1 = z;
      for (int k = 2; k <= m; ++k) {
        ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = (m == 1) ? 1 : m * (z * p1 - p0) / (z * z - 1);
    }
    x[m - 1 - i] = z / 2;
    w[m - 1 - i] = 1 / ((1 - z * z) * dp * dp);
  }
  for (int i = 0; i < m / 2; ++i) {      // exact antisymmetry of the nodes
    ld a = (x[m - 1 - i] - x[i]) / 2;
    x[i] = -a;
    x[m - 1 - i] = a;
    ld ww = (w[i] + w[m - 1 - i]) / 2;
    w[i] = w[m - 1 - i] = ww;
  }
  if (m % 2) x[m / 2] = 0;
}

// ---------------------------------------------------------------------------
// 1D cell-average -> point weights on cells s0 .. s0+k-1 (unit cells, target
// cell [-1/2, 1/2]).  Built from the primitive function: U is interpolated
// at the k+1 cell interfaces by the Lagrange polynomial and p = U', so the
// weight of cell i is the sum of L_e'(xi) over the interfaces e to its right.
// ---------------------------------------------------------------------------
void weights_1d(int s0, int k, ld xi, ld* w) {
  std::vector<ld> xe(k + 1), dl(k + 1);
  for (int e = 0; e <= k; ++e) xe[e] = s0 - 0.5L + e;
  for (int e = 0; e <= k; ++e) {
    ld sum = 0;
    for (int l = 0; l <= k; ++l) {
      if (l == e) continue;
      ld prod = 1 / (xe[e] - xe[l]);
      for (int nn = 0; nn <= k; ++nn) {
        if (nn == e || nn == l) continue;
        prod *= (xi - xe[nn]) / (xe[e] - xe[nn]);
      }
      sum += prod;
    }
    dl[e] = sum;
  }
  for (int i = 0; i < k; ++i) {
    ld acc = 0;
    for (int e = i + 1; e <= k; ++e) acc += dl[e];
    w[i] = acc;
  }
}

// 1D linear weights d_s of WENO of order n = 2l-1 at xi: sum_s d_s w_s = w_H,
// solved by substitution from whichever end has the larger pivots.
bool linear_weights_1d(int l, ld xi, ld* d) {
  int n = 2 * l - 1;
  std::vector<ld> H(n), Ws(l * l);
  weights_1d(-(l - 1), n, xi, H.data());
  for (int s = 0; s < l; ++s) weights_1d(s - (l - 1), l, xi, &Ws[s * l]);
  std::vector<ld> dl(l), dr(l);
  ld pl = 1e300L, pr = 1e300L;
  for (int c = 0; c < l; ++c) {     // from the left: cell c is covered by sub-stencils s <= c
    ld acc = H[c];
    for (int s = 0; s < c; ++s) acc -= dl[s] * Ws[s * l + (c - s)];
    ld piv = Ws[c * l + 0];
    pl = std::min(pl, std::fabs(piv));
    dl[c] = acc / piv;
  }
  for (int c = n - 1; c >= n - l; --c) {   // from the right
    int s = c - (l - 1);
    ld acc = H[c];
    for (int s2 = s + 1; s2 < l; ++s2) acc -= dr[s2] * Ws[s2 * l + (c - s2)];
    ld piv = Ws[s * l + (l - 1)];
    pr = std::min(pr, std::fabs(piv));
    dr[s] = acc / piv;
  }
  const std::vector<ld>& dd = (pl >= pr) ? dl : dr;
  for (int s = 0; s < l; ++s) d[s] = dd[s];
  // residual of all n equations
  ld res = 0;
  for (int c = 0; c < n; ++c) {
    ld acc = -H[c];
    for (int s = 0; s < l; ++s)
      if (c >= s && c < s + l) acc += d[s] * Ws[s * l + (c - s)];
    res = std::max(res, std::fabs(acc));
  }
  return res < 1e-14L;
}

// Symmetric eigen-decomposition by cyclic Jacobi rotations (small matrices).
void jacobi_eigen(int n, std::vector<ld>& A, std::vector<ld>& V, std::vector<ld>& ev) {
  V.assign(n * n, 0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1;
  for (int sweep = 0; sweep < 100; ++sweep) {
    ld off = 0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
    if (off < 1e-38L) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        ld apq = A[p * n + q];
        if (std::fabs(apq) < 1e-40L) continue;
        ld theta = (A[q * n + q] - A[p * n + p]) / (2 * apq);
        ld t = (theta >= 0 ? 1 : -1) / (std::fabs(theta) + std::sqrt(theta * theta + 1));
        ld c = 1 / std::sqrt(t * t + 1), s = t * c;
        for (int k = 0; k < n; ++k) {
          ld akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          ld apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          ld vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  ev.resize(n);
  for (int i = 0; i < n; ++i) ev[i] = A[i * n + i];
}

// Smoothness-indicator tables.  The indicator of a sub-stencil polynomial p
// is the sum over derivative orders (a, b) != (0, 0), a, b < l, of the
// integral over the unit target cell of (d^a_x d^b_y p)^2.  With the 1D
// Gram matrices K_a (derivative order a, monomial basis) and S = sum_a K_a,
// choose the basis phi_alpha orthonormal for K_0 that diagonalises S
// (S phi = s phi); then in the product basis the indicator is
// sum_{alpha,beta} c_{alpha beta}^2 (s_alpha s_beta - 1), with the constant
// mode (s = 1) dropping out.  c = V_sy (x) V_sx applied to the cell averages,
// V_s[alpha][o] = integral of phi_alpha(xi) w_o(xi) over the target cell.
void smoothness_tables(int l, std::vector<double>& Vout, std::vector<double>& lamout) {
  auto moment = [](int p) -> ld { return (p % 2) ? 0 : 2.0L / ((p + 1) * std::pow(2.0L, p + 1)); };
  auto dco = [](int al, int a) -> ld {
    if (a > al) return 0;
    ld c = 1;
    for (int t = 0; t < a; ++t) c *= (al - t);
    return c;
  };
  std::vector<ld> K0(l * l), S(l * l, 0);
  for (int a = 0; a < l; ++a)
    for (int i = 0; i < l; ++i)
      for (int j = 0; j < l; ++j) {
        ld v = (i >= a && j >= a) ? dco(i, a) * dco(j, a) * moment(i + j - 2 * a) : 0;
        S[i * l + j] += v;
        if (a == 0) K0[i * l + j] = v;
      }
  // Cholesky K0 = L L^T
  std::vector<ld> L(l * l, 0);
  for (int i = 0; i < l; ++i)
    for (int j = 0; j <= i; ++j) {
      ld s = K0[i * l + j];
      for (int k = 0; k < j; ++k) s -= L[i * l + k] * L[j * l + k];
      L[i * l + j] = (i == j) ? std::sqrt(s) : s / L[j * l + j];
    }
  // Li = L^{-1}
  std::vector<ld> Li(l * l, 0);
  for (int c = 0; c < l; ++c)
    for (int i = 0; i < l; ++i) {
      ld s = (i == c) ? 1 : 0;
      for (int k = 0; k < i; ++k) s -= L[i * l + k] * Li[k * l + c];
      Li[i * l + c] = s / L[i * l + i];
    }
  // M = Li S Li^T
  std::vector<ld> M(l * l, 0);
  for (int i = 0; i < l; ++i)
    for (int j = 0; j < l; ++j) {
      ld s = 0;
      for (int a = 0; a < l; ++a)
        for (int b = 0; b < l; ++b) s += Li[i * l + a] * S[a * l + b] * Li[j * l + b];
      M[i * l + j] = s;
    }
  std::vector<ld> Y, ev;
  jacobi_eigen(l, M, Y, ev);
  // Phi = Li^T Y : column alpha holds the monomial coefficients of phi_alpha
  std::vector<ld> Phi(l * l, 0);
  for (int j = 0; j < l; ++j)
    for (int al = 0; al < l; ++al) {
      ld s = 0;
      for (int i = 0; i < l; ++i) s += Li[i * l + j] * Y[i * l + al];
      Phi[j * l + al] = s;
    }
  // order: ascending eigenvalue (the constant mode, s = 1, first)
  std::vector<int> ord(l);
  for (int i = 0; i < l; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return ev[a] < ev[b]; });
  // V_s[alpha][o] by Gauss quadrature (exact: degree <= 2l-2)
  std::vector<ld> gx, gwt;
  gauss_rule(l + 1, gx, gwt);
  std::vector<ld> Vacc(l * l * l, 0);
  for (int st = 0; st < l; ++st) {
    int s0 = st - (l - 1);
    for (int q = 0; q <= l; ++q) {
      std::vector<ld> w(l);
      weights_1d(s0, l, gx[q], w.data());
      for (int a = 0; a < l; ++a) {
        int al = ord[a];
        ld phi = 0, xp = 1;
        for (int j = 0; j < l; ++j) { phi += Phi[j * l + al] * xp; xp *= gx[q]; }
        for (int o = 0; o < l; ++o) Vacc[(st * l + a) * l + o] += gwt[q] * phi * w[o];
      }
    }
  }
  Vout.assign(l * l * l, 0);
  for (size_t i = 0; i < Vacc.size(); ++i) Vout[i] = (double)Vacc[i];
  lamout.assign(l * l, 0);
  for (int b = 0; b < l; ++b)
    for (int a = 0; a < l; ++a) lamout[b * l + a] = (double)(ev[ord[a]] * ev[ord[b]] - 1);
  lamout[0] = 0;   // the constant mode carries no smoothness
}

// ---------------------------------------------------------------------------
// Cube geometry, built from 3D basis vectors
// ---------------------------------------------------------------------------
// unnormalised direction of (X, Y) on panel p, and its X- and Y-derivatives
void panel_vec(int p, ld X, ld Y, ld v[3], ld dX[3], ld dY[3]) {
  ld t[6][9] = {
      {1, X, Y, 0, 1, 0, 0, 0, 1},     {-X, 1, Y, -1, 0, 0, 0, 0, 1}, {-1, -X, Y, 0, -1, 0, 0, 0, 1},
      {X, -1, Y, 1, 0, 0, 0, 0, 1},    {-Y, X, 1, 0, 1, 0, -1, 0, 0}, {Y, X, -1, 0, 1, 0, 1, 0, 0}};
  for (int c = 0; c < 3; ++c) {
    v[c] = t[p][c];
    dX[c] = t[p][3 + c];
    dY[c] = t[p][6 + c];
  }
}

void inverse_map(int p, const ld u[3], ld& X, ld& Y) {
  ld a = u[0], b = u[1], c = u[2];
  switch (p) {
    case 0: X = b / a; Y = c / a; break;
    case 1: X = -a / b; Y = c / b; break;
    case 2: X = b / a; Y = -c / a; break;
    case 3: X = -a / b; Y = -c / b; break;
    case 4: X = b / c; Y = -a / c; break;
    default: X = -b / c; Y = -a / c; break;
  }
}

// covariant basis e_x, e_y (3D, on the sphere of radius a) at (X, Y) of panel p
void basis(int p, ld X, ld Y, ld a, ld ex[3], ld ey[3]) {
  ld v[3], dX[3], dY[3];
  panel_vec(p, X, Y, v, dX, dY);
  ld d2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  ld d = std::sqrt(d2);
  ld vdx = v[0] * dX[0] + v[1] * dX[1] + v[2] * dX[2];
  ld vdy = v[0] * dY[0] + v[1] * dY[1] + v[2] * dY[2];
  for (int c = 0; c < 3; ++c) {
    ex[c] = a * (1 + X * X) * (dX[c] / d - v[c] * vdx / (d * d2));
    ey[c] = a * (1 + Y * Y) * (dY[c] / d - v[c] * vdy / (d * d2));
  }
}

ld dot3(const ld* a, const ld* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Conversion of (sqrtG phi, sqrtG phi u, sqrtG phi v) from panel B to panel A at
// one point: mass ratio sqrtG_A / sqrtG_B and C = ratio * (grad x_A^i . e_B_j).
void conversion(int A, ld XA, ld YA, int B, ld XB, ld YB, ld a, ld out[5]) {
  ld eA[2][3], eB[2][3];
  basis(A, XA, YA, a, eA[0], eA[1]);
  basis(B, XB, YB, a, eB[0], eB[1]);
  ld gA[4] = {dot3(eA[0], eA[0]), dot3(eA[0], eA[1]), dot3(eA[1], eA[0]), dot3(eA[1], eA[1])};
  ld gB[4] = {dot3(eB[0], eB[0]), dot3(eB[0], eB[1]), dot3(eB[1], eB[0]), dot3(eB[1], eB[1])};
  ld detA = gA[0] * gA[3] - gA[1] * gA[2];
  ld detB = gB[0] * gB[3] - gB[1] * gB[2];
  ld ratio = std::sqrt(detA) / std::sqrt(detB);
  ld iA[4] = {gA[3] / detA, -gA[1] / detA, -gA[2] / detA, gA[0] / detA};
  ld m[4];   // (e_A_i . e_B_j)
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) m[i * 2 + j] = dot3(eA[i], eB[j]);
  out[0] = ratio;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      out[1 + i * 2 + j] = ratio * (iA[i * 2 + 0] * m[0 * 2 + j] + iA[i * 2 + 1] * m[1 * 2 + j]);
}

const int kAxisDir[6][3] = {{1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

// owner panel(s) of a direction: largest signed component; tie within 1e-12
int owners(const ld u[3], int& second, bool& tie) {
  ld c[6];
  for (int p = 0; p < 6; ++p) c[p] = kAxisDir[p][0] * u[0] + kAxisDir[p][1] * u[1] + kAxisDir[p][2] * u[2];
  int b = 0;
  for (int p = 1; p < 6; ++p)
    if (c[p] > c[b]) b = p;
  int s = (b == 0) ? 1 : 0;
  for (int p = 0; p < 6; ++p)
    if (p != b && c[p] > c[s]) s = p;
  second = s;
  tie = std::fabs(c[b] - c[s]) <= 1e-12L * std::fabs(c[b]);
  return b;
}

void unit_vec(int p, ld X, ld Y, ld u[3]) {
  ld v[3], dX[3], dY[3];
  panel_vec(p, X, Y, v, dX, dY);
  ld d = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  for (int c = 0; c < 3; ++c) u[c] = v[c] / d;
}

// ---------------------------------------------------------------------------
// Ghost map: sparse rows (same pattern for mass and momentum blocks)
// ---------------------------------------------------------------------------
struct Entry {
  int32_t col;
  double v[5];
};

// iters = 0: the fixed point G = Lq + Lg G of the ghost interpolation, by
// Gauss-Seidel sweeps over sparse rows until converged; iters = N > 0: the
// map of exactly N Jacobi sweeps from g = 0 (G_1 = Lq, G_{s+1} = Lq + Lg G_s),
// the truncated map the paper builds with its 10 sweeps
int build_ghost_map(HostTables& t, int iters) {
  const int n = t.n, k = t.k, r = t.r, P = t.P, m = t.m;
  const ld D = kPi / (2 * (ld)n);
  std::vector<ld> gx, gwt;
  gauss_rule(m, gx, gwt);
  const int plane = 6 * P * P;
  std::vector<int32_t> gidx(plane, -1);
  std::vector<int32_t> dst;
  for (int A = 0; A < 6; ++A)
    for (int jj = 0; jj < P; ++jj)
      for (int ii = 0; ii < P; ++ii) {
        bool inner = jj >= r && jj < r + n && ii >= r && ii < r + n;
        if (inner) continue;
        int off = A * P * P + jj * P + ii;
        gidx[off] = (int32_t)dst.size();
        dst.push_back(off);
      }
  const int G = (int)dst.size();
  // local operator: for each ghost row, (col, coef[5], is_ghost)
  std::vector<std::vector<Entry>> Lq(G), Lg(G);
  std::vector<ld> wx(k), wy(k);
  for (int g = 0; g < G; ++g) {
    int off = dst[g];
    int A = off / (P * P), jj = (off / P) % P, ii = off % P;
    std::vector<std::pair<int32_t, std::array<ld, 5>>> acc;   // unsorted, merged later
    for (int hy = 0; hy < m; ++hy)
      for (int hx = 0; hx < m; ++hx) {
        ld x = ((ld)(ii - r) + 0.5L - n / 2.0L + gx[hx]) * D;
        ld y = ((ld)(jj - r) + 0.5L - n / 2.0L + gx[hy]) * D;
        ld XA = std::tan(x), YA = std::tan(y);
        ld u[3];
        unit_vec(A, XA, YA, u);
        int second;
        bool tie;
        int best = owners(u, second, tie);
        for (int br = 0; br < (tie ? 2 : 1); ++br) {
          int B = br == 0 ? best : second;
          ld fac = tie ? 0.5L : 1.0L;
          ld XB, YB;
          inverse_map(B, u, XB, YB);
          ld xb = std::atan(XB), yb = std::atan(YB);
          int ib = (int)std::floor(xb / D + n / 2.0L), jb = (int)std::floor(yb / D + n / 2.0L);
          ib = std::min(std::max(ib, 0), n - 1);
          jb = std::min(std::max(jb, 0), n - 1);
          ld xi = xb / D - (ib + 0.5L - n / 2.0L), eta = yb / D - (jb + 0.5L - n / 2.0L);
          weights_1d(-r, k, xi, wx.data());
          weights_1d(-r, k, eta, wy.data());
          ld cv[5];
          conversion(A, XA, YA, B, XB, YB, t.radius, cv);
          ld q = gwt[hx] * gwt[hy] * fac;
          for (int b = 0; b < k; ++b)
            for (int a = 0; a < k; ++a) {
              ld w = q * wy[b] * wx[a];
              int32_t col = B * P * P + (jb + b) * P + (ib + a);
              std::array<ld, 5> e = {w * cv[0], w * cv[1], w * cv[2], w * cv[3], w * cv[4]};
              acc.push_back({col, e});
            }
        }
      }
    std::sort(acc.begin(), acc.end(), [](auto& a, auto& b) { return a.first < b.first; });
    for (size_t i = 0; i < acc.size();) {
      size_t j = i;
      std::array<ld, 5> s = {0, 0, 0, 0, 0};
      while (j < acc.size() && acc[j].first == acc[i].first) {
        for (int c = 0; c < 5; ++c) s[c] += acc[j].second[c];
        ++j;
      }
      Entry e;
      e.col = acc[i].first;
      for (int c = 0; c < 5; ++c) e.v[c] = (double)s[c];
      if (gidx[e.col] >= 0) {
        e.col = gidx[e.col];
        Lg[g].push_back(e);
      } else {
        Lq[g].push_back(e);
      }
      i = j;
    }
  }
  // Fixed point G = Lq + Lg (x) G by Gauss-Seidel sweeps on sparse rows.
  std::vector<std::vector<Entry>> Gm(G);
  for (int g = 0; g < G; ++g) Gm[g] = Lq[g];
  std::vector<double> dense(5 * (size_t)plane, 0.0);
  std::vector<int32_t> touched;
  std::vector<char> mark(plane, 0);
  int sweeps = 0, settle = -1;
  const bool jacobi = iters > 0;
  std::vector<std::vector<Entry>> prev;   // the previous sweep's rows (Jacobi)
  for (; sweeps < 300; ++sweeps) {
    if (jacobi) {
      if (sweeps + 1 >= iters) break;     // G_1 = Lq is the first sweep
      prev = Gm;
    }
    const std::vector<std::vector<Entry>>& src = jacobi ? prev : Gm;
    double maxrel = 0;
    for (int g = 0; g < G; ++g) {
      touched.clear();
      auto add = [&](int32_t col, const double* v) {
        if (!mark[col]) { mark[col] = 1; touched.push_back(col); }
        for (int c = 0; c < 5; ++c) dense[5 * (size_t)col + c] += v[c];
      };
      for (const Entry& e : Lq[g]) add(e.col, e.v);
      for (const Entry& ref : Lg[g]) {
        const double* c = ref.v;
        for (const Entry& e : src[ref.col]) {
          double v[5];
          v[0] = c[0] * e.v[0];
          v[1] = c[1] * e.v[1] + c[2] * e.v[3];
          v[2] = c[1] * e.v[2] + c[2] * e.v[4];
          v[3] = c[3] * e.v[1] + c[4] * e.v[3];
          v[4] = c[3] * e.v[2] + c[4] * e.v[4];
          add(e.col, v);
        }
      }
      std::sort(touched.begin(), touched.end());
      double rowmax = 0;
      for (int32_t col : touched)
        for (int c = 0; c < 5; ++c) rowmax = std::max(rowmax, std::fabs(dense[5 * (size_t)col + c]));
      std::vector<Entry> row;
      row.reserve(touched.size());
      for (int32_t col : touched) {
        Entry e;
        e.col = col;
        double mx = 0;
        for (int c = 0; c < 5; ++c) {
          e.v[c] = dense[5 * (size_t)col + c];
          mx = std::max(mx, std::fabs(e.v[c]));
          dense[5 * (size_t)col + c] = 0;
        }
        mark[col] = 0;
        if (mx > 1e-18 * rowmax) row.push_back(e);
      }
      // change against the previous row (both sorted by column)
      const std::vector<Entry>& old = Gm[g];
      size_t a = 0, b = 0;
      double diff = 0;
      while (a < old.size() || b < row.size()) {
        if (b >= row.size() || (a < old.size() && old[a].col < row[b].col)) {
          for (int c = 0; c < 5; ++c) diff = std::max(diff, std::fabs(old[a].v[c]));
          ++a;
        } else if (a >= old.size() || row[b].col < old[a].col) {
          for (int c = 0; c < 5; ++c) diff = std::max(diff, std::fabs(row[b].v[c]));
          ++b;
        } else {
          for (int c = 0; c < 5; ++c) diff = std::max(diff, std::fabs(row[b].v[c] - old[a].v[c]));
          ++a;
          ++b;
        }
      }
      maxrel = std::max(maxrel, diff / (rowmax > 0 ? rowmax : 1));
      Gm[g].swap(row);
    }
    if (jacobi) continue;
    if (settle < 0 && maxrel < 1e-15) settle = 2;
    if (settle >= 0) {
      if (settle == 0) { ++sweeps; break; }
      --settle;
    }
  }
  if (!jacobi && settle != 0 && sweeps >= 300) {
    t.error = "ghost map fixed point did not converge";
    return HOPE_ERR_NUMERIC;
  }
  t.ghost_sweeps = jacobi ? iters : sweeps;
  // final drop: entries below 1e-16 of the row's largest entry
  t.g_dst.assign(dst.begin(), dst.end());
  t.g_ptr.assign(G + 1, 0);
  std::vector<int32_t> cols;
  std::vector<double> vals[5];
  for (int g = 0; g < G; ++g) {
    double rowmax = 0;
    for (const Entry& e : Gm[g])
      for (int c = 0; c < 5; ++c) rowmax = std::max(rowmax, std::fabs(e.v[c]));
    for (const Entry& e : Gm[g]) {
      double mx = 0;
      for (int c = 0; c < 5; ++c) mx = std::max(mx, std::fabs(e.v[c]));
      if (mx < 1e-16 * rowmax) continue;
      // interior column: padded offset within one plane
      cols.push_back(e.col);
      for (int c = 0; c < 5; ++c) vals[c].push_back(e.v[c]);
    }
    t.g_ptr[g + 1] = (int32_t)cols.size();
  }
  t.g_col = cols;
  size_t nnz = cols.size();
  t.g_val.resize(5 * nnz);
  for (int c = 0; c < 5; ++c) std::copy(vals[c].begin(), vals[c].end(), t.g_val.begin() + c * nnz);
  return 0;
}

// ---------------------------------------------------------------------------
// Rotation compression of the ghost map.  Each of the cube's 24 rotations maps
// panels onto panels and, on each panel, the gnomonic coordinates (X, Y) by a
// signed permutation (a frame code, see GhostDev).  The rotations act freely on
// ghost cells, and the quarter of panel 0's ghost ring below its bottom edge
// (padded rows 0..r-1, padded columns 0..n+r-1) meets every orbit once, so
// every ghost row is the image of one such canonical row: the same mass
// weights at the image cells, and momentum blocks T(f_ghost) C T(f_cell)^T.
// The map built by the fixed point is checked against its images (they agree
// to rounding) and then replaced by them, so that the rows the host reports,
// the adjoint's transpose and the compressed device rows are one map.
// ---------------------------------------------------------------------------
namespace {

struct CubeRot {
  int img[6];    // image panel of each panel
  int code[6];   // frame code on each panel
};

// frame code f: (X, Y) -> (sx (sw ? Y : X), sy (sw ? X : Y))
void frame_apply(int f, ld X, ld Y, ld& X2, ld& Y2) {
  const bool sw = f & 1;
  const ld sx = (f & 2) ? -1 : 1, sy = (f & 4) ? -1 : 1;
  X2 = sx * (sw ? Y : X);
  Y2 = sy * (sw ? X : Y);
}

// the same on centred cell indices i in [-r, n+r) (X -> -X is i -> n-1-i)
void frame_index(int f, int n, int i, int j, int& i2, int& j2) {
  const bool sw = f & 1;
  const int a = sw ? j : i, b = sw ? i : j;
  i2 = (f & 2) ? n - 1 - a : a;
  j2 = (f & 4) ? n - 1 - b : b;
}

// 2x2 matrix of a frame code acting on contravariant components
void frame_matrix(int f, ld T[4]) {
  const bool sw = f & 1;
  const ld sx = (f & 2) ? -1 : 1, sy = (f & 4) ? -1 : 1;
  T[0] = sw ? 0 : sx;
  T[1] = sw ? sx : 0;
  T[2] = sw ? sy : 0;
  T[3] = sw ? 0 : sy;
}

int cube_rotations(std::vector<CubeRot>& out, std::string& err) {
  const int perms[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {0, 2, 1}, {2, 1, 0}, {1, 0, 2}};
  const int psign[6] = {1, 1, 1, -1, -1, -1};
  const ld pts[2][2] = {{0.3L, 0.1L}, {-0.2L, 0.45L}};
  for (int pi = 0; pi < 6; ++pi)
    for (int sg = 0; sg < 8; ++sg) {
      const int sgn[3] = {(sg & 1) ? -1 : 1, (sg & 2) ? -1 : 1, (sg & 4) ? -1 : 1};
      if (psign[pi] * sgn[0] * sgn[1] * sgn[2] != 1) continue;   // proper rotations only
      auto rot = [&](const ld u[3], ld u2[3]) {
        for (int c = 0; c < 3; ++c) u2[c] = sgn[c] * u[perms[pi][c]];
      };
      CubeRot R;
      for (int B = 0; B < 6; ++B) {
        ld a[3] = {(ld)kAxisDir[B][0], (ld)kAxisDir[B][1], (ld)kAxisDir[B][2]}, a2[3];
        rot(a, a2);
        R.img[B] = -1;
        for (int B2 = 0; B2 < 6; ++B2)
          if (kAxisDir[B2][0] == (int)a2[0] && kAxisDir[B2][1] == (int)a2[1] && kAxisDir[B2][2] == (int)a2[2])
            R.img[B] = B2;
        R.code[B] = -1;
        for (int f = 0; f < 8 && R.code[B] < 0; ++f) {
          bool ok = true;
          for (const auto& pt : pts) {
            ld u[3], u2[3], X2, Y2, eX, eY;
            unit_vec(B, pt[0], pt[1], u);
            rot(u, u2);
            inverse_map(R.img[B], u2, X2, Y2);
            frame_apply(f, pt[0], pt[1], eX, eY);
            ok = ok && std::fabs(X2 - eX) < 1e-12L && std::fabs(Y2 - eY) < 1e-12L;
          }
          if (ok) R.code[B] = f;
        }
        if (R.img[B] < 0 || R.code[B] < 0) {
          err = "cube rotation does not map panel coordinates by a signed permutation";
          return HOPE_ERR_NUMERIC;
        }
      }
      out.push_back(R);
    }
  if (out.size() != 24) {
    err = "cube rotation group incomplete";
    return HOPE_ERR_NUMERIC;
  }
  return 0;
}

}  // namespace

int compress_ghost_map(HostTables& t) {
  const int n = t.n, r = t.r, P = t.P;
  const int PP = P * P;
  std::vector<CubeRot> rots;
  if (int st = cube_rotations(rots, t.error)) return st;
  const int G = (int)t.g_dst.size();
  std::vector<int32_t> gidx(6 * (size_t)PP, -1);
  for (int g = 0; g < G; ++g) gidx[t.g_dst[g]] = g;
  // image of a padded offset under rotation R
  auto image = [&](const CubeRot& R, int32_t off) {
    const int B = off / PP, jj = (off / P) % P, ii = off % P;
    int i2, j2;
    frame_index(R.code[B], n, ii - r, jj - r, i2, j2);
    return (int32_t)(R.img[B] * PP + (j2 + r) * P + (i2 + r));
  };
  struct E {
    int32_t col;
    int canon;    // entry within the canonical row
    int code;     // frame code on the cell's panel
    double v[5];
  };
  const size_t nnz = t.g_col.size();
  std::vector<int32_t> hit(G, 0);
  std::vector<std::vector<E>> rows(G);     // symmetrised rows, by ghost row index
  std::vector<int> row_canon(G), row_code(G), row_rot(G), canon_start;
  std::vector<int32_t> canon_rows;         // row index of each canonical ghost
  for (int jj = 0; jj < r; ++jj)
    for (int ii = 0; ii < n + r; ++ii) canon_rows.push_back(gidx[jj * P + ii]);
  if ((int)canon_rows.size() * 24 != G) {
    t.error = "ghost rows are not 24 copies of the canonical rows";
    return HOPE_ERR_NUMERIC;
  }
  std::vector<double> cval[5];
  double worst = 0;
  for (size_t c = 0; c < canon_rows.size(); ++c) {
    const int g0 = canon_rows[c];
    if (g0 < 0) {
      t.error = "canonical ghost cell missing";
      return HOPE_ERR_NUMERIC;
    }
    const int32_t b = t.g_ptr[g0], e = t.g_ptr[g0 + 1];
    canon_start.push_back((int)cval[0].size());
    for (int32_t k = b; k < e; ++k)
      for (int comp = 0; comp < 5; ++comp) cval[comp].push_back(t.g_val[comp * nnz + k]);
    for (int ri = 0; ri < 24; ++ri) {
      const CubeRot& R = rots[ri];
      const int32_t d = image(R, t.g_dst[g0]);
      const int g = gidx[d];
      if (g < 0 || hit[g]++) {
        t.error = "rotation images of the ghost ring do not tile it";
        return HOPE_ERR_NUMERIC;
      }
      row_canon[g] = (int)c;
      row_rot[g] = ri;
      const int f0 = R.code[0];
      row_code[g] = f0;
      ld T0[4];
      frame_matrix(f0, T0);
      std::vector<E>& row = rows[g];
      row.reserve(e - b);
      for (int32_t k = b; k < e; ++k) {
        E x;
        x.col = image(R, t.g_col[k]);
        x.canon = k - b;
        x.code = R.code[t.g_col[k] / PP];
        ld T[4];
        frame_matrix(x.code, T);
        const ld C[4] = {t.g_val[nnz + k], t.g_val[2 * nnz + k], t.g_val[3 * nnz + k], t.g_val[4 * nnz + k]};
        ld TC[4];   // T0 C
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j) TC[i * 2 + j] = T0[i * 2] * C[j] + T0[i * 2 + 1] * C[2 + j];
        x.v[0] = t.g_val[k];
        for (int i = 0; i < 2; ++i)       // (T0 C) T^T; exact, T and T0 are signed permutations
          for (int j = 0; j < 2; ++j) x.v[1 + i * 2 + j] = (double)(TC[i * 2] * T[j * 2] + TC[i * 2 + 1] * T[j * 2 + 1]);
        row.push_back(x);
      }
      std::sort(row.begin(), row.end(), [](const E& a, const E& b2) { return a.col < b2.col; });
      // agreement with the row the fixed point gave for this ghost
      double rowmax = 0, diff = 0;
      const int32_t ob = t.g_ptr[g], oe = t.g_ptr[g + 1];
      for (int32_t k = ob; k < oe; ++k)
        for (int comp = 0; comp < 5; ++comp) rowmax = std::max(rowmax, std::fabs(t.g_val[comp * nnz + k]));
      size_t a = 0;
      int32_t k = ob;
      while (a < row.size() || k < oe) {
        if (k >= oe || (a < row.size() && row[a].col < t.g_col[k])) {
          for (int comp = 0; comp < 5; ++comp) diff = std::max(diff, std::fabs(row[a].v[comp]));
          ++a;
        } else if (a >= row.size() || t.g_col[k] < row[a].col) {
          for (int comp = 0; comp < 5; ++comp) diff = std::max(diff, std::fabs(t.g_val[comp * nnz + k]));
          ++k;
        } else {
          for (int comp = 0; comp < 5; ++comp)
            diff = std::max(diff, std::fabs(row[a].v[comp] - t.g_val[comp * nnz + k]));
          ++a;
          ++k;
        }
      }
      worst = std::max(worst, diff / (rowmax > 0 ? rowmax : 1));
      if (e - b >= (1 << 13)) {
        t.error = "ghost row longer than 8191 entries";
        return HOPE_ERR_UNSUPPORTED;
      }
    }
  }
  if (worst > 1e-12) {
    char buf[128];
    std::snprintf(buf, sizeof buf, "ghost map not rotation symmetric (max relative difference %.3g)", worst);
    t.error = buf;
    return HOPE_ERR_NUMERIC;
  }
  // the host rows become the symmetrised ones (same row order)
  std::vector<int32_t> ptr(G + 1, 0), col;
  std::vector<double> val[5];
  for (int g = 0; g < G; ++g) {
    for (const E& x : rows[g]) {
      col.push_back(x.col);
      for (int comp = 0; comp < 5; ++comp) val[comp].push_back(x.v[comp]);
    }
    ptr[g + 1] = (int32_t)col.size();
  }
  t.g_ptr = ptr;
  t.g_col = col;
  t.g_val.resize(5 * col.size());
  for (int comp = 0; comp < 5; ++comp) std::copy(val[comp].begin(), val[comp].end(), t.g_val.begin() + comp * col.size());
  // device form.  Row order: the canonical strip (r deep, n+r long) is cut
  // along its length into kXcdChunks spans; rows go by span, then rotation,
  // then position along the edge and depth.  Neighbouring rows read
  // overlapping stencils, and the ghost-fill kernels give each of the chip's
  // 8 L2 domains one contiguous range of rows, so each touches about one
  // span's canonical values and ghost stencils rather than all of them.
  const size_t cnnz = cval[0].size();
  if (cnnz >= (size_t)1 << 28) {
    t.error = "canonical ghost map too large";
    return HOPE_ERR_UNSUPPORTED;
  }
  t.z_cval.assign(6 * cnnz, 0.0);
  for (size_t e = 0; e < cnnz; ++e)
    for (int comp = 0; comp < 5; ++comp) t.z_cval[6 * e + comp] = cval[comp][e];
  t.z_dst.clear();
  t.z_info.clear();
  t.z_ent.clear();
  t.z_ptr.assign(1, 0);
  const int L = n + r, kXcdChunks = 8;
  std::vector<int> order(G);
  std::vector<int64_t> key(G);
  for (int g = 0; g < G; ++g) {
    const int ii = row_canon[g] % L, jj = row_canon[g] / L;
    key[g] = (((int64_t)(ii * kXcdChunks / L) * 24 + row_rot[g]) * L + ii) * r + jj;
    order[g] = g;
  }
  std::sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
  for (int g : order) {
    t.z_dst.push_back(t.g_dst[g]);
    t.z_info.push_back(canon_start[row_canon[g]] | (row_code[g] << 28));
    for (const E& x : rows[g]) {
      t.z_ent.push_back(x.col);
      t.z_ent.push_back(x.canon | (x.code << 13));
    }
    t.z_ptr.push_back((int32_t)(t.z_ent.size() / 2));
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Panel-edge trace maps: the neighbour cell and Gauss point at every EQP of
// every panel side, and the conversion into this panel's variables.
// ---------------------------------------------------------------------------
int build_edge_maps(HostTables& t) {
  const int n = t.n, r = t.r, P = t.P, m = t.m;
  const ld D = kPi / (2 * (ld)n);
  std::vector<ld> gx, gwt;
  gauss_rule(m, gx, gwt);
  t.bt_cell.assign(24 * n, 0);
  t.bt_side.assign(24 * n, 0);
  t.bt_rev.assign(24 * n, 0);
  t.bt_conv.assign(24 * (size_t)n * m * 5, 0);
  for (int A = 0; A < 6; ++A)
    for (int side = 0; side < 4; ++side) {
      ld sgn = (side == 0 || side == 2) ? -1 : 1;
      ld out = std::tan(sgn * (kPi / 4 + D / 2));
      ld uo[3];
      if (side < 2) unit_vec(A, out, 0, uo); else unit_vec(A, 0, out, uo);
      int second;
      bool tie;
      int B = owners(uo, second, tie);
      for (int tt = 0; tt < n; ++tt) {
        int bside = -1, bidx = -1, rev = 0;
        for (int h = 0; h < m; ++h) {
          ld along = std::tan(((ld)tt + 0.5L - n / 2.0L + gx[h]) * D);
          ld XA = side < 2 ? sgn : along, YA = side < 2 ? along : sgn;
          ld u[3];
          unit_vec(A, XA, YA, u);
          ld XB, YB;
          inverse_map(B, u, XB, YB);
          int bs;
          ld alongB;
          if (std::fabs(std::fabs(XB) - 1) < 1e-9L) { bs = XB < 0 ? 0 : 1; alongB = std::atan(YB); }
          else if (std::fabs(std::fabs(YB) - 1) < 1e-9L) { bs = YB < 0 ? 2 : 3; alongB = std::atan(XB); }
          else { t.error = "panel edge point not on a neighbour edge"; return HOPE_ERR_NUMERIC; }
          int ib = (int)std::floor(alongB / D + n / 2.0L);
          ib = std::min(std::max(ib, 0), n - 1);
          ld loc = alongB / D - (ib + 0.5L - n / 2.0L);
          int hb = -1;
          for (int q = 0; q < m; ++q)
            if (std::fabs(loc - gx[q]) < 1e-9L) hb = q;
          if (hb < 0) { t.error = "panel edge Gauss points do not match"; return HOPE_ERR_NUMERIC; }
          if (h == 0) { bside = bs; bidx = ib; rev = (m > 1 && hb == m - 1) ? 1 : 0; }
          if (bs != bside || ib != bidx || hb != (rev ? m - 1 - h : h)) {
            t.error = "inconsistent panel edge map";
            return HOPE_ERR_NUMERIC;
          }
          // the EQP lies exactly on the edge in both panels
          ld XBe = XB, YBe = YB;
          if (bs < 2) XBe = bs == 0 ? -1 : 1; else YBe = bs == 2 ? -1 : 1;
          ld cv[5];
          conversion(A, XA, YA, B, XBe, YBe, t.radius, cv);
          size_t o = (((size_t)(A * 4 + side) * n + tt) * m + h) * 5;
          for (int c = 0; c < 5; ++c) t.bt_conv[o + c] = (double)cv[c];
        }
        int ib = bside < 2 ? (bside == 0 ? 0 : n - 1) : bidx;
        int jb = bside < 2 ? bidx : (bside == 2 ? 0 : n - 1);
        int idx = (A * 4 + side) * n + tt;
        t.bt_cell[idx] = B * P * P + (jb + r) * P + (ib + r);
        t.bt_side[idx] = bside;
        t.bt_rev[idx] = rev;
      }
    }
  return 0;
}

}  // namespace

int build_tables(HostTables& t, int n, int k, int weno, double radius, double omega, double tilt,
                 double eps, double theta, int ghost_iters) {
  t.n = n;
  t.k = k;
  t.r = (k - 1) / 2;
  t.m = (k + 1) / 2;
  t.P = n + 2 * t.r;
  t.weno = weno;
  t.radius = radius;
  t.omega = omega;
  t.tilt = tilt;
  t.eps = eps;
  t.theta = theta;
  t.delta = (double)(kPi / (2 * (ld)n));
  const int m = t.m, k2 = k;
  std::vector<ld> gx, gwt;
  gauss_rule(m, gx, gwt);
  t.gnode.resize(m);
  t.gw.resize(m);
  for (int i = 0; i < m; ++i) { t.gnode[i] = (double)gx[i]; t.gw[i] = (double)gwt[i]; }
  std::vector<ld> axis(2 + m);
  axis[0] = -0.5L;
  axis[1] = 0.5L;
  for (int i = 0; i < m; ++i) axis[2 + i] = gx[i];
  t.wc.resize((2 + m) * k2);
  for (int a = 0; a < 2 + m; ++a) {
    std::vector<ld> w(k2);
    weights_1d(-t.r, k2, axis[a], w.data());
    for (int i = 0; i < k2; ++i) t.wc[a * k2 + i] = (double)w[i];
  }
  if (weno) {
    const int l = (k + 1) / 2, s = l * l, npts = 4 * m + m * m;
    t.l = l;
    t.s = s;
    t.wsub.resize(l * (2 + m) * l);
    std::vector<ld> d((2 + m) * l);
    for (int st = 0; st < l; ++st)
      for (int a = 0; a < 2 + m; ++a) {
        std::vector<ld> w(l);
        weights_1d(st - (l - 1), l, axis[a], w.data());
        for (int i = 0; i < l; ++i) t.wsub[(st * (2 + m) + a) * l + i] = (double)w[i];
      }
    for (int a = 0; a < 2 + m; ++a)
      if (!linear_weights_1d(l, axis[a], &d[a * l])) {
        t.error = "WENO linear weights: no exact solution";
        return HOPE_ERR_NUMERIC;
      }
    t.d1.resize((2 + m) * l);
    for (int a = 0; a < 2 + m; ++a) {
      bool neg = false;
      for (int i = 0; i < l; ++i) {
        t.d1[a * l + i] = (double)d[a * l + i];
        neg = neg || d[a * l + i] < 0;
      }
      if (neg != weno_mixed_axis(k, m, a)) {
        t.error = "WENO linear weights: sign pattern differs from the one the kernels are built for";
        return HOPE_ERR_NUMERIC;
      }
    }
    // point order: x-edge left (h), x-edge right (h), y-edge bottom (h), y-edge top (h), CQP (v outer, h inner)
    auto pt_axes = [&](int pt, int& ax, int& ay) {
      if (pt < m) { ax = 0; ay = 2 + pt; }
      else if (pt < 2 * m) { ax = 1; ay = 2 + pt - m; }
      else if (pt < 3 * m) { ax = 2 + pt - 2 * m; ay = 0; }
      else if (pt < 4 * m) { ax = 2 + pt - 3 * m; ay = 1; }
      else { int c = pt - 4 * m; ax = 2 + c % m; ay = 2 + c / m; }
    };
    t.gp.resize(npts * s);
    t.gm.resize(npts * s);
    t.sp.resize(npts);
    t.sm.resize(npts);
    for (int pt = 0; pt < npts; ++pt) {
      int ax, ay;
      pt_axes(pt, ax, ay);
      ld sp = 0, sm = 0;
      for (int sy = 0; sy < l; ++sy)
        for (int sx = 0; sx < l; ++sx) {
          ld g = d[ay * l + sy] * d[ax * l + sx];
          ld gp = ((ld)theta * std::fabs(g) + g) / 2, gmv = ((ld)theta * std::fabs(g) - g) / 2;
          t.gp[pt * s + sy * l + sx] = (double)gp;
          t.gm[pt * s + sy * l + sx] = (double)gmv;
          sp += gp;
          sm += gmv;
        }
      t.sp[pt] = (double)sp;
      t.sm[pt] = (double)sm;
    }
    smoothness_tables(l, t.V, t.lam);
  }
  // metric tables
  t.Xe.resize(n + 1);
  for (int e = 0; e <= n; ++e) t.Xe[e] = (double)std::tan(((ld)e - n / 2.0L) * (ld)kPi / (2 * (ld)n));
  t.Xe[0] = -1.0;
  t.Xe[n] = 1.0;
  t.Xg.resize(n * m);
  for (int i = 0; i < n; ++i)
    for (int h = 0; h < m; ++h)
      t.Xg[i * m + h] = (double)std::tan(((ld)i + 0.5L - n / 2.0L + gx[h]) * kPi / (2 * (ld)n));
  t.sqe.resize(n + 1);
  for (int e = 0; e <= n; ++e) {
    ld X = (e == 0) ? -1 : (e == n) ? 1 : std::tan(((ld)e - n / 2.0L) * (ld)kPi / (2 * (ld)n));
    t.sqe[e] = (double)std::sqrt(1 + X * X);
  }
  t.sqg.resize(n * m);
  for (int i = 0; i < n; ++i)
    for (int h = 0; h < m; ++h) {
      ld X = std::tan(((ld)i + 0.5L - n / 2.0L + gx[h]) * kPi / (2 * (ld)n));
      t.sqg[i * m + h] = (double)std::sqrt(1 + X * X);
    }
  t.fcoef.resize(18);
  coriolis_coefs(tilt, t.fcoef.data());
  int st = build_ghost_map(t, ghost_iters);
  if (!st) st = compress_ghost_map(t);
  if (st) return st;
  return build_edge_maps(t);
}

// d/dxi of the centred weights of order k at the 2+m axis points (x-edges,
// Gauss nodes), out[a*k + i]: the primitive U is the Lagrange interpolant of
// the interfaces, p = U', so dp/dxi = U'' and cell i's weight is the sum of
// L_e''(xi) over the interfaces e to its right.
void derivative_weights(int k, int m, std::vector<double>& out) {
  std::vector<ld> gx, gwt;
  gauss_rule(m, gx, gwt);
  std::vector<ld> axis(2 + m);
  axis[0] = -0.5L;
  axis[1] = 0.5L;
  for (int i = 0; i < m; ++i) axis[2 + i] = gx[i];
  const int r = (k - 1) / 2;
  std::vector<ld> xe(k + 1), d2(k + 1);
  for (int e = 0; e <= k; ++e) xe[e] = -r - 0.5L + e;
  out.assign((2 + m) * k, 0.0);
  for (int a = 0; a < 2 + m; ++a) {
    const ld xi = axis[a];
    for (int e = 0; e <= k; ++e) {
      ld sum = 0;
      for (int l = 0; l <= k; ++l) {
        if (l == e) continue;
        for (int q = 0; q <= k; ++q) {
          if (q == e || q == l) continue;
          ld prod = 1 / ((xe[e] - xe[l]) * (xe[e] - xe[q]));
          for (int o = 0; o <= k; ++o) {
            if (o == e || o == l || o == q) continue;
            prod *= (xi - xe[o]) / (xe[e] - xe[o]);
          }
          sum += prod;
        }
      }
      d2[e] = sum;
    }
    for (int i = 0; i < k; ++i) {
      ld acc = 0;
      for (int e = i + 1; e <= k; ++e) acc += d2[e];
      out[a * k + i] = (double)acc;
    }
  }
}

// ---------------------------------------------------------------------------
// Bottom topography (section 2, (2.13)-(2.14)).  The kernels reconstruct the
// mass as sqrtG phi_t = sqrtG phi + sqrtG phi_s: they add the cell averages
// of sqrtG phi_s (ghost cells: the ghost map applied to them, as to any
// reconstruction variable) before reconstructing, and subtract the point
// values of sqrtG phi_s at every edge and cell Gauss point afterwards.
// ---------------------------------------------------------------------------
int build_topography(const HostTables& t, SurfaceFn fn, void* user, TopoHost& out, std::string& err) {
  const int n = t.n, m = t.m, P = t.P, r = t.r;
  const ld a = t.radius;
  auto sg_at = [&](ld X, ld Y) {
    const ld d2 = 1 + X * X + Y * Y;
    return a * a * (1 + X * X) * (1 + Y * Y) / (d2 * std::sqrt(d2));
  };
  std::vector<double> xyz, val;
  // phi_s at npt points of panel p given by coords(i, X, Y)
  auto eval = [&](int p, size_t npt, auto coords, auto store) -> bool {
    xyz.resize(3 * npt);
    val.assign(npt, std::numeric_limits<double>::quiet_NaN());
    std::vector<ld> XX(npt), YY(npt);
    for (size_t i = 0; i < npt; ++i) {
      coords(i, XX[i], YY[i]);
      ld u[3];
      unit_vec(p, XX[i], YY[i], u);
      for (int c = 0; c < 3; ++c) xyz[3 * i + c] = (double)u[c];
    }
    fn((int64_t)npt, xyz.data(), val.data(), user);
    for (size_t i = 0; i < npt; ++i) {
      if (!std::isfinite(val[i])) {
        err = "surface_geopotential returned a value that is not finite";
        return false;
      }
      store(i, sg_at(XX[i], YY[i]) * (ld)val[i]);
    }
    return true;
  };
  // cell averages over dx dy by an nq x nq Gauss rule
  constexpr int nq = 4;
  std::vector<ld> qx, qw;
  gauss_rule(nq, qx, qw);
  const ld h = kPi / (2 * (ld)n);
  out.sbar.assign(6 * (size_t)P * P, 0.0);
  std::vector<ld> acc((size_t)n * n);
  for (int p = 0; p < 6; ++p) {
    std::fill(acc.begin(), acc.end(), 0.0L);
    const size_t npt = (size_t)n * n * nq * nq;
    auto coords = [&](size_t idx, ld& X, ld& Y) {
      const size_t cell = idx / (nq * nq);
      const int q = (int)(idx % (nq * nq));
      const int i = (int)(cell % n), j = (int)(cell / n);
      X = std::tan((i + 0.5L - n / 2.0L + qx[q % nq]) * h);
      Y = std::tan((j + 0.5L - n / 2.0L + qx[q / nq]) * h);
    };
    auto store = [&](size_t idx, ld v) {
      const int q = (int)(idx % (nq * nq));
      acc[idx / (nq * nq)] += qw[q % nq] * qw[q / nq] * v;
    };
    if (!eval(p, npt, coords, store)) return HOPE_ERR_INVALID;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i)
        out.sbar[((size_t)p * P + j + r) * P + i + r] = (double)acc[(size_t)j * n + i];
  }
  for (size_t row = 0; row + 1 < t.g_ptr.size(); ++row) {
    ld s = 0;
    for (int32_t k = t.g_ptr[row]; k < t.g_ptr[row + 1]; ++k) s += (ld)t.g_val[k] * out.sbar[t.g_col[k]];
    out.sbar[t.g_dst[row]] = (double)s;
  }
  // point values at the edge and cell Gauss points
  out.sx.assign(6 * (size_t)n * (n + 1) * m, 0.0);
  out.sy.assign(6 * (size_t)(n + 1) * n * m, 0.0);
  out.sc.assign(6 * (size_t)n * n * m * m, 0.0);
  for (int p = 0; p < 6; ++p) {
    double* sx = out.sx.data() + (size_t)p * n * (n + 1) * m;
    auto cx = [&](size_t idx, ld& X, ld& Y) {        // [j][i][h], i = edge 0..n
      const int hh = (int)(idx % m), i = (int)((idx / m) % (n + 1)), j = (int)(idx / (m * (n + 1)));
      X = t.Xe[i];
      Y = t.Xg[j * m + hh];
    };
    if (!eval(p, (size_t)n * (n + 1) * m, cx, [&](size_t idx, ld v) { sx[idx] = (double)v; })) return HOPE_ERR_INVALID;
    double* sy = out.sy.data() + (size_t)p * (n + 1) * n * m;
    auto cy = [&](size_t idx, ld& X, ld& Y) {        // [j][i][h], j = edge 0..n
      const int hh = (int)(idx % m), i = (int)((idx / m) % n), j = (int)(idx / (m * n));
      X = t.Xg[i * m + hh];
      Y = t.Xe[j];
    };
    if (!eval(p, (size_t)(n + 1) * n * m, cy, [&](size_t idx, ld v) { sy[idx] = (double)v; })) return HOPE_ERR_INVALID;
    double* sc = out.sc.data() + (size_t)p * n * n * m * m;
    auto cc = [&](size_t idx, ld& X, ld& Y) {        // [j][i][w][h]
      const int hh = (int)(idx % m), w = (int)((idx / m) % m), i = (int)((idx / (m * m)) % n),
                j = (int)(idx / ((size_t)m * m * n));
      X = t.Xg[i * m + hh];
      Y = t.Xg[j * m + w];
    };
    if (!eval(p, (size_t)n * n * m * m, cc, [&](size_t idx, ld v) { sc[idx] = (double)v; })) return HOPE_ERR_INVALID;
  }
  return HOPE_OK;
}

// Coriolis parameter on panel p: f = 2 Omega (Omega_hat . p_hat) with the axis
const char* tables_build_stamp() { return "host tables " __DATE__ " " __TIME__; }

// tilted by alpha towards -x, Omega_hat = (-sin alpha, 0, cos alpha).  With the
// unnormalised panel point v = (c0 + X cX + Y cY per component), Omega_hat . v =
// L0 + LX X + LY Y; out[3p..3p+2] = (L0, LX, LY).
void coriolis_coefs(double tilt, double* out) {
  ld sa = std::sin((ld)tilt), ca = std::cos((ld)tilt);
  const ld fc[6][3] = {{-sa, 0, ca}, {0, sa, ca}, {sa, 0, ca}, {0, -sa, ca}, {ca, 0, sa}, {-ca, 0, -sa}};
  for (int p = 0; p < 6; ++p)
    for (int c = 0; c < 3; ++c) out[p * 3 + c] = (double)fc[p][c];
}

}  // namespace hope
