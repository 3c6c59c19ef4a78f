"""Pins of the oracle's reconstruction weights, Gauss rules and WENO tables
against exact mathematics and textbook values (sections 3.1-3.2)."""
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

from oracle import weights as W


@pytest.mark.parametrize("k", [3, 5, 7, 9, 11, 13])
def test_1d_weights_reproduce_polynomials(k):
    """A degree < k polynomial's cell averages reconstruct its exact point value
    (the defining property of (3.11)-(3.14), checked without the inverse)."""
    offs = W.centred(k)
    rng = np.random.default_rng(k)
    for xi in list(rng.uniform(-0.5, 0.5, 5)) + [-0.5, 0.5]:
        w = W.weights_1d_mp(offs, mp.mpf(float(xi)))
        for j in range(k):
            avg = [mp.mpf(W.cell_moment(o, j).numerator) / W.cell_moment(o, j).denominator for o in offs]
            val = mp.fsum(wi * a for wi, a in zip(w, avg))
            assert abs(val - mp.mpf(float(xi)) ** j) < mp.mpf(10) ** -35


def test_1d_textbook_edge_weights():
    """Third- and fifth-order cell-average -> interface values (WENO literature)."""
    w3 = W.recon_poly_1d((-1, 0, 1))
    val3 = [sum(c * Fraction(1, 2) ** j for j, c in enumerate(row)) for row in w3]
    assert val3 == [Fraction(-1, 6), Fraction(5, 6), Fraction(1, 3)]
    w5 = W.recon_poly_1d((-2, -1, 0, 1, 2))
    val5 = [sum(c * Fraction(1, 2) ** j for j, c in enumerate(row)) for row in w5]
    assert val5 == [Fraction(2, 60), Fraction(-13, 60), Fraction(47, 60), Fraction(27, 60), Fraction(-3, 60)]


@pytest.mark.parametrize("k", [3, 5])
def test_separable_tpp_equals_literal_2d_solve(k):
    """The tensor-product form used everywhere equals R = C A^-1 (3.15) solved
    literally on the k^2 x k^2 moment matrix, in exact rationals."""
    pts = [(Fraction(1, 2), Fraction(1, 7)), (Fraction(-1, 2), Fraction(-2, 5)), (Fraction(1, 3), Fraction(1, 2)),
           (Fraction(0), Fraction(0))]
    R = W.tpp_2d_matrix_rational(k, pts)
    offs = W.centred(k)
    for (x, y), row in zip(pts, R):
        wx = [sum(c * x ** j for j, c in enumerate(r)) for r in W.recon_poly_1d(offs)]
        wy = [sum(c * y ** j for j, c in enumerate(r)) for r in W.recon_poly_1d(offs)]
        sep = [wy[b] * wx[a] for b in range(k) for a in range(k)]
        assert sep == row


def test_f64_weights_match_multiprecision():
    for k in (3, 5, 11, 13):
        xs = np.random.default_rng(1).uniform(-0.5, 0.5, 50)
        a = W.weights_1d_f64(W.centred(k), xs)
        b = np.array([[float(v) for v in W.weights_1d_mp(W.centred(k), mp.mpf(float(x)))] for x in xs])
        assert np.abs(a - b).max() < 4e-16


@pytest.mark.parametrize("m", [1, 2, 3, 4, 6, 7, 8])
def test_gauss_rule_exact_to_degree_2m_minus_1(m):
    nodes, wts = W.gauss_mp(m)
    for deg in range(2 * m):
        exact = mp.mpf(0) if deg % 2 else mp.mpf(2) / ((deg + 1) * mp.mpf(2) ** (deg + 1))
        assert abs(mp.fsum(w * x ** deg for x, w in zip(nodes, wts)) - exact) < mp.mpf(10) ** -40
    ref, _ = np.polynomial.legendre.leggauss(m)
    assert np.allclose(np.array([float(v) for v in nodes]), np.sort(ref) / 2, atol=1e-15)


def _d1(n, xi):
    """1D linear weights of n-th order WENO at xi, solved from the 1D system
    sum_s d_s w_s(xi) = w_H(xi) (the 1D analogue of (3.17))."""
    l = (n + 1) // 2
    H = W.weights_1d_mp(W.centred(n), xi)
    subs = [tuple(range(s, s + l)) for s in range(-(l - 1), 1)]
    M = mp.matrix(n, l)
    for j, s in enumerate(subs):
        ws = W.weights_1d_mp(s, xi)
        for a, o in enumerate(s):
            M[o + (n - 1) // 2, j] = ws[a]
    return mp.lu_solve(M.T * M, M.T * mp.matrix(H))


@pytest.mark.parametrize("n,m", [(3, 2), (5, 3)])
def test_weno_linear_weights(n, m):
    """(3.19): residual-free least squares, weights sum to one, and equal the
    tensor product of the 1D linear weights."""
    gam, res = W.weno_linear_weights(n, m)
    assert res.max() < 1e-40
    assert np.allclose(gam.sum(1), 1.0, atol=1e-15)
    pts = W.cell_points_mp(m)
    for g, (xi, eta) in zip(gam, pts):
        dx, dy = _d1(n, xi), _d1(n, eta)
        l = (n + 1) // 2
        tp = np.array([float(dy[b] * dx[a]) for b in range(l) for a in range(l)])
        assert np.allclose(g, tp, atol=1e-15)


def test_weno_textbook_1d_weights():
    half = mp.mpf(1) / 2
    assert np.allclose([float(v) for v in _d1(3, half)], [1 / 3, 2 / 3], atol=1e-15)
    assert np.allclose([float(v) for v in _d1(5, half)], [0.1, 0.6, 0.3], atol=1e-15)
    assert np.allclose([float(v) for v in _d1(5, mp.mpf(0))], [-9 / 80, 49 / 40, -9 / 80], atol=1e-15)
    assert np.allclose([float(v) for v in _d1(3, -mp.sqrt(3) / 6)], [0.5, 0.5], atol=1e-15)


def test_split_weights():
    g = np.array([[-0.1, 0.6, 0.5]])
    gp, gm, sp, sm = W.split_weights(g)
    assert np.allclose(gp - gm, g) and (gp >= 0).all() and (gm >= 0).all()
    assert np.allclose(sp - sm, 1.0)


@pytest.mark.parametrize("k", [2, 3, 4, 5, 7, 11, 13])
def test_weights_mirror_symmetry(k):
    """Reflecting x -> -x maps a stencil S to -S and its cell o to -o, so the
    weight of cell o of S at xi equals the weight of cell -o of -S at -xi:
    as polynomials in xi, c_S[o][j] (-1)^j = c_{-S}[-o][j], exactly.  Checked
    for every sub-stencil of width k that contains the target cell."""
    for start in range(-(k - 1), 1):
        offs = tuple(range(start, start + k))
        mirror = tuple(sorted(-o for o in offs))
        c, cm = W.recon_poly_1d(offs), W.recon_poly_1d(mirror)
        for oi, o in enumerate(offs):
            mi = mirror.index(-o)
            assert [cj * (-1) ** j for j, cj in enumerate(c[oi])] == list(cm[mi])
