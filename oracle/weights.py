"""Reconstruction weights, Gauss rules, WENO linear weights and smoothness
indicator forms, built exactly (rationals) or in high precision (mpmath) and
rounded to FP64 once.  Test infrastructure only (see the package docstring).

Coordinates are the paper's unit-cell coordinates (section 3.1, text after
(3.9)): the target cell is [-1/2, 1/2]^2 and cell o of a stencil is
[o-1/2, o+1/2] along each axis.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache

import mpmath as mp
import numpy as np

mp.mp.dps = 50


# ----------------------------------------------------------------------------
# Exact linear algebra in rationals
# ----------------------------------------------------------------------------
def frac_inverse(M):
    """Gauss-Jordan inverse of a square matrix of Fractions."""
    n = len(M)
    A = [list(row) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(M)]
    for c in range(n):
        piv = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[piv] = A[piv], A[c]
        inv = 1 / A[c][c]
        A[c] = [v * inv for v in A[c]]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c]
                A[r] = [a - f * b for a, b in zip(A[r], A[c])]
    return [row[n:] for row in A]


def cell_moment(o: int, j: int) -> Fraction:
    """Integral of x^j over the unit cell [o-1/2, o+1/2]  (the entries of psi_i, (3.10))."""
    a = Fraction(2 * o - 1, 2)
    b = Fraction(2 * o + 1, 2)
    return (b ** (j + 1) - a ** (j + 1)) / (j + 1)


# ----------------------------------------------------------------------------
# 1D building block: cell averages on consecutive cells -> value at xi
# ----------------------------------------------------------------------------
@lru_cache(maxsize=None)
def recon_poly_1d(offsets: tuple) -> tuple:
    """Coefficients c[o][j] with w_o(xi) = sum_j c[o][j] xi^j.

    For the 1D polynomial basis x^j, j < k, the moment system A a = qbar
    ((3.11)-(3.12) in one dimension) is solved exactly, a = A^-1 qbar
    (3.13), and the point value c(xi)^T A^-1 qbar (3.14) gives the weights.
    """
    k = len(offsets)
    A = [[cell_moment(o, j) for j in range(k)] for o in offsets]
    Ainv = frac_inverse(A)
    return tuple(tuple(Ainv[j][oi] for j in range(k)) for oi in range(k))


def weights_1d_mp(offsets, xi) -> list:
    """Weights at one point in mpmath (xi may be an mpf or a Fraction)."""
    coef = recon_poly_1d(tuple(offsets))
    x = mp.mpf(xi) if not isinstance(xi, Fraction) else mp.mpf(xi.numerator) / xi.denominator
    out = []
    for row in coef:
        v = mp.mpf(0)
        for c in reversed(row):
            v = v * x + mp.mpf(c.numerator) / c.denominator
        out.append(v)
    return out


def weights_1d_f64(offsets, xi) -> np.ndarray:
    """Weights at many points xi (float array) -> (..., k) float64.

    Horner evaluation in extended precision (numpy longdouble) of the exact
    rational coefficients, rounded once to FP64.
    """
    coef = recon_poly_1d(tuple(offsets))
    x = np.asarray(xi, dtype=np.longdouble)
    out = []
    for row in coef:
        v = np.zeros_like(x)
        for c in reversed(row):
            v = v * x + (np.longdouble(c.numerator) / np.longdouble(c.denominator))
        out.append(v)
    return np.stack(out, axis=-1).astype(np.float64)


def centred(k: int) -> tuple:
    r = (k - 1) // 2
    return tuple(range(-r, r + 1))


# ----------------------------------------------------------------------------
# Brute-force 2D TPP (3.7)-(3.15) in rationals: pins the separable form
# ----------------------------------------------------------------------------
def tpp_2d_matrix_rational(k: int, points) -> list:
    """Literal R = C A^-1 (3.15) on the centred k x k stencil.

    The basis c_k(x, y) = x^alpha y^beta, alpha, beta < k ((3.7)); stencil
    cells ordered row by row (y outer, x inner); points are (xi, eta)
    rational pairs.  Returns a list of rows (one per point) of k*k Fractions.
    """
    offs = centred(k)
    cells = [(ox, oy) for oy in offs for ox in offs]
    terms = [(al, be) for be in range(k) for al in range(k)]
    A = [[cell_moment(ox, al) * cell_moment(oy, be) for (al, be) in terms] for (ox, oy) in cells]
    Ainv = frac_inverse(A)
    rows = []
    for (x, y) in points:
        c = [Fraction(x) ** al * Fraction(y) ** be for (al, be) in terms]
        rows.append([sum(c[t] * Ainv[t][ci] for t in range(len(terms))) for ci in range(len(cells))])
    return rows


# ----------------------------------------------------------------------------
# Gauss-Legendre on [-1/2, 1/2]  ((3.5), (3.6))
# ----------------------------------------------------------------------------
@lru_cache(maxsize=None)
def gauss_mp(m: int):
    """m-point Gauss-Legendre nodes and weights on [-1/2, 1/2] (weights sum to 1).

    Newton iteration on the Legendre polynomial in 50-digit arithmetic,
    started from numpy's nodes; nodes are made exactly antisymmetric.
    """
    x0, _ = np.polynomial.legendre.leggauss(m)
    nodes, wts = [], []
    for x in x0:
        x = mp.mpf(float(x))
        for _ in range(100):
            p = mp.legendre(m, x)
            dp = m * (x * p - mp.legendre(m - 1, x)) / (x * x - 1)
            dx = p / dp
            x -= dx
            if abs(dx) < mp.mpf(10) ** (-45):
                break
        dp = m * (x * mp.legendre(m, x) - mp.legendre(m - 1, x)) / (x * x - 1)
        nodes.append(x / 2)
        wts.append(1 / ((1 - x * x) * dp * dp))   # 2/((1-x^2)P'^2) halved
    order = sorted(range(m), key=lambda i: nodes[i])
    nodes = [nodes[i] for i in order]
    wts = [wts[i] for i in order]
    for i in range(m // 2):
        a = (nodes[m - 1 - i] - nodes[i]) / 2
        nodes[i], nodes[m - 1 - i] = -a, a
        w = (wts[i] + wts[m - 1 - i]) / 2
        wts[i] = wts[m - 1 - i] = w
    if m % 2:
        nodes[m // 2] = mp.mpf(0)
    return tuple(nodes), tuple(wts)


def gauss(m: int):
    n, w = gauss_mp(m)
    return np.array([float(v) for v in n]), np.array([float(v) for v in w])


# ----------------------------------------------------------------------------
# Point sets of one cell (Figure 3.2)
# ----------------------------------------------------------------------------
def edge_points_mp(m: int):
    """1D coordinates used by the reconstruction along one axis.

    Returns the list [-1/2, +1/2, g_1 .. g_m]: the two edges and the m
    Gauss nodes.  An EQP on an x-edge is (edge, g_h); on a y-edge (g_h, edge);
    a CQP is (g_h, g_v).
    """
    nodes, _ = gauss_mp(m)
    return [mp.mpf(-1) / 2, mp.mpf(1) / 2] + list(nodes)


@lru_cache(maxsize=None)
def axis_weights(offsets: tuple, m: int) -> np.ndarray:
    """(2+m, k) FP64 weights of a stencil at the 2+m axis coordinates."""
    return np.array([[float(v) for v in weights_1d_mp(offsets, x)] for x in edge_points_mp(m)])


def derivative_weights_1d_mp(offsets, xi) -> list:
    """d/dxi of the weights of weights_1d_mp at xi (mpmath): the derivative
    of the reconstruction polynomial (3.14) at xi from the cell averages."""
    coef = recon_poly_1d(tuple(offsets))
    x = mp.mpf(xi) if not isinstance(xi, Fraction) else mp.mpf(xi.numerator) / xi.denominator
    out = []
    for row in coef:
        v = mp.mpf(0)
        for j in range(len(row) - 1, 0, -1):
            v = v * x + j * mp.mpf(row[j].numerator) / row[j].denominator
        out.append(v)
    return out


@lru_cache(maxsize=None)
def axis_derivative_weights(offsets: tuple, m: int) -> np.ndarray:
    """(2+m, k) FP64 derivative weights of a stencil at the 2+m axis coordinates."""
    return np.array([[float(v) for v in derivative_weights_1d_mp(offsets, x)] for x in edge_points_mp(m)])


# ----------------------------------------------------------------------------
# Genuine 2D WENO: linear weights by least squares (3.16)-(3.20)
# ----------------------------------------------------------------------------
def substencil_offsets(n: int):
    """The s = l^2 sub-stencils of an n x n stencil (Figs 3.4-3.5).

    Sub-stencil j covers x offsets sx..sx+l-1 and y offsets sy..sy+l-1,
    sx, sy in {-(l-1), .., 0}; ordered with sy outer, sx inner.
    """
    l = (n + 1) // 2
    starts = list(range(-(l - 1), 1))
    return [(sx, sy) for sy in starts for sx in starts]


def tpp_row_mp(xoffs, yoffs, xi, eta):
    """One row of the TPP reconstruction matrix on an arbitrary rectangular
    stencil at (xi, eta), in mpmath, cells ordered (y outer, x inner).

    Uses the factorisation of the TPP moment matrix into x and y parts: for
    the basis x^a y^b the moment of a unit cell is the product of the 1D
    moments, so A = A_y (x) A_x and R = (c_y A_y^-1) (x) (c_x A_x^-1).
    The brute-force test checks this against the literal 2D solve.
    """
    wx = weights_1d_mp(tuple(xoffs), xi)
    wy = weights_1d_mp(tuple(yoffs), eta)
    return [wy[b] * wx[a] for b in range(len(yoffs)) for a in range(len(xoffs))]


@lru_cache(maxsize=None)
def weno_linear_weights(n: int, m: int):
    """Optimal linear weights gamma at every point of a cell, by (3.19).

    For each point (xi, eta) of the point set (x-edge EQPs, y-edge EQPs,
    CQPs, see ``cell_points``) builds R_H (1 x n^2), the extended sub-stencil
    rows R_Li = R_i E (1 x n^2), solves the normal equations of
    R_L gamma = R_H in 50-digit arithmetic and returns
    (gamma (P, s), residual (P,)) in FP64.
    """
    full = centred(n)
    subs = substencil_offsets(n)
    l = (n + 1) // 2
    pts = cell_points_mp(m)
    gam, res = [], []
    for (xi, eta) in pts:
        RH = tpp_row_mp(full, full, xi, eta)
        cols = []
        for (sx, sy) in subs:
            xo = tuple(range(sx, sx + l))
            yo = tuple(range(sy, sy + l))
            Ri = tpp_row_mp(xo, yo, xi, eta)
            # extension E: place sub-stencil cell (a, b) at its position in the big stencil
            ext = [mp.mpf(0)] * (n * n)
            for b in range(l):
                for a in range(l):
                    ext[(yo[b] - full[0]) * n + (xo[a] - full[0])] = Ri[b * l + a]
            cols.append(ext)
        RL = mp.matrix(n * n, len(subs))
        for j, c in enumerate(cols):
            for i in range(n * n):
                RL[i, j] = c[i]
        rh = mp.matrix(RH)
        g = mp.lu_solve(RL.T * RL, RL.T * rh)
        r = RL * g - rh
        gam.append([float(g[j]) for j in range(len(subs))])
        res.append(float(mp.norm(r)))
    return np.array(gam), np.array(res)


def split_weights(gamma: np.ndarray, theta: float = 3.0):
    """(3.20): gamma+- = (theta|gamma| +- gamma)/2 and sigma+- = sum gamma+-."""
    gp = (theta * np.abs(gamma) + gamma) / 2
    gm = (theta * np.abs(gamma) - gamma) / 2
    return gp, gm, gp.sum(-1), gm.sum(-1)


def cell_points_mp(m: int):
    """All reconstruction points of a cell, in this order:

    x-edge EQPs: (-1/2, g_h) h=0..m-1, then (+1/2, g_h);
    y-edge EQPs: (g_h, -1/2), then (g_h, +1/2);
    CQPs: (g_h, g_v) with v outer, h inner.
    """
    nodes, _ = gauss_mp(m)
    half = mp.mpf(1) / 2
    pts = [(-half, g) for g in nodes] + [(half, g) for g in nodes]
    pts += [(g, -half) for g in nodes] + [(g, half) for g in nodes]
    pts += [(gh, gv) for gv in nodes for gh in nodes]
    return pts


def cell_points(m: int) -> np.ndarray:
    return np.array([[float(a), float(b)] for a, b in cell_points_mp(m)])


# ----------------------------------------------------------------------------
# Smoothness indicators (3.25)
# ----------------------------------------------------------------------------
@lru_cache(maxsize=None)
def substencil_poly_1d(l: int, start: int):
    """Exact 1D coefficient matrix (l x l): coefficient j of the polynomial
    from the cell averages of cells start..start+l-1 is sum_o M[j][o] qbar_o."""
    coef = recon_poly_1d(tuple(range(start, start + l)))
    return [[coef[o][j] for o in range(l)] for j in range(l)]


@lru_cache(maxsize=None)
def derivative_gram(l: int):
    """K[a][al][al2] = integral over [-1/2,1/2] of D^a x^al * D^a x^al2 (exact)."""
    def dcoef(al, a):
        if a > al:
            return 0
        c = 1
        for t in range(a):
            c *= (al - t)
        return c

    def moment(p):
        if p % 2:
            return Fraction(0)
        return Fraction(2, (p + 1) * 2 ** (p + 1))

    K = []
    for a in range(l):
        Ka = [[Fraction(dcoef(al, a) * dcoef(al2, a)) * (moment(al + al2 - 2 * a) if al >= a and al2 >= a else 0)
               for al2 in range(l)] for al in range(l)]
        K.append(Ka)
    return K
