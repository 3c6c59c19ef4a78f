"""Exact pins of the oracle's genuine 2D WENO nonlinear weighting (section
3.2, (3.20)-(3.25)) and of the LMARS jump terms ((3.32)-(3.33)), on inputs
small enough to work out by hand, and planted slips that show each pin fails
on the mistakes it guards against.

The expected values come by routes other than the oracle's:
  * WENO3: a sub-stencil polynomial of degree <= 1 in each variable has cell
    averages equal to its values at the cell centres, so it is the bilinear
    interpolant of the four centre values; its smoothness indicator is then
    a three-term closed form (below).
  * WENO5: on additively separable data a(x) + b(y) every sub-stencil
    polynomial is P(x) + Q(y), its mixed derivatives vanish, and the 2D
    indicator of (3.25) is the sum of the two 1D indicators, which are the
    classical fifth-order Jiang-Shu indicators (13/12 and 1/4 forms).
  * Linear weights: the textbook 1D values, multiplied (gamma = d(eta) d(xi)).
  * Sub-stencil point values: the textbook 1D cell-average -> point formulas.
Only the WENO-Z combination itself, (3.20)-(3.24), is restated here; its
inputs are not the oracle's, and tau is also checked against a number worked
out by hand.
"""
import inspect
import math
import textwrap
from fractions import Fraction as Fr

import mpmath as mp
import numpy as np
import pytest
import torch

import oracle.rhs as orhs
from oracle import geometry as geo
from oracle.rhs import Grid, WenoTables

A = 6.371e6


# ----------------------------------------------------------------------------
# WENO-Z combination (3.20)-(3.23), exact (Fractions / mpmath)
# ----------------------------------------------------------------------------
def wenoz_value(gammas, betas, tau, p_vals, eps=Fr(0), theta=3):
    """sigma+ sum w+ p - sigma- sum w- p with gamma+- = (theta|gamma| +- gamma)/2,
    alpha+- = gamma+- (1 + tau/(beta + eps)), w+- = alpha+- / sum alpha+-."""
    gp = [(theta * abs(g) + g) / 2 for g in gammas]
    gm = [(theta * abs(g) - g) / 2 for g in gammas]
    kap = [1 + tau / (b + eps) for b in betas]
    ap = [g * k for g, k in zip(gp, kap)]
    am = [g * k for g, k in zip(gm, kap)]
    sp, sm = sum(gp), sum(gm)
    vp = mp.fsum(mp.mpf(a.numerator) / a.denominator * p for a, p in zip(ap, p_vals)) / (
        mp.mpf(sum(ap).numerator) / sum(ap).denominator)
    out = mp.mpf(sp.numerator) / sp.denominator * vp
    if sm:
        vm = mp.fsum(mp.mpf(a.numerator) / a.denominator * p for a, p in zip(am, p_vals)) / (
            mp.mpf(sum(am).numerator) / sum(am).denominator)
        out -= mp.mpf(sm.numerator) / sm.denominator * vm
    return out


# ----------------------------------------------------------------------------
# WENO3 worked example (n = 3, l = 2, s = 4)
# ----------------------------------------------------------------------------
D3 = [[1, 0, 2],       # row y = -1, columns x = -1, 0, 1
      [3, 1, 5],       # row y =  0
      [0, 4, 2]]       # row y = +1
SUBS3 = [(-1, -1), (0, -1), (-1, 0), (0, 0)]     # oracle order: sy outer, sx inner


def d3(x, y):
    return D3[y + 1][x + 1]


def bilinear3(sx, sy):
    """p = v00 + b (x - sx) + c (y - sy) + d (x - sx)(y - sy) through the four
    centre values of the sub-stencil with lower-left cell (sx, sy)."""
    v00, v10, v01, v11 = d3(sx, sy), d3(sx + 1, sy), d3(sx, sy + 1), d3(sx + 1, sy + 1)
    return v00, v10 - v00, v01 - v00, v11 - v10 - v01 + v00


def beta3_closed_form(sx, sy):
    """(3.25) for the bilinear p over the target cell [-1/2, 1/2]^2:
    int p_x^2 = (b - d sy)^2 + d^2/12, int p_y^2 = (c - d sx)^2 + d^2/12,
    int p_xy^2 = d^2, so beta = (b - d sy)^2 + (c - d sx)^2 + 7/6 d^2."""
    _, b, c, d = bilinear3(sx, sy)
    return Fr(b - d * sy) ** 2 + Fr(c - d * sx) ** 2 + Fr(7, 6) * d * d


# by hand: (b, c, d) = (-1, 2, -1), (2, 1, 2), (-2, -3, 6), (4, 3, -6) for the
# four sub-stencils in oracle order, so beta = 4 + 1 + 7/6, 16 + 1 + 14/3,
# 4 + 9 + 42 and 16 + 9 + 42
BCD3 = [(-1, 2, -1), (2, 1, 2), (-2, -3, 6), (4, 3, -6)]
BETA3 = [Fr(37, 6), Fr(65, 3), Fr(55), Fr(67)]
# |differences| of the 6 pairs: 31/2, 293/6, 365/6, 100/3, 136/3, 12 -> 1295/6;
# tau = 2/(4*5) * 1295/6
TAU3 = Fr(259, 12)


def test_weno3_beta_and_tau_worked_example():
    assert [bilinear3(sx, sy)[1:] for sx, sy in SUBS3] == BCD3
    assert [beta3_closed_form(sx, sy) for sx, sy in SUBS3] == BETA3
    wt = WenoTables(3, 2, eps=0.0)
    q = torch.tensor(np.array(D3, dtype=np.float64))
    beta = wt.beta(q, 1).reshape(-1)
    for got, want in zip(beta.tolist(), BETA3):
        assert abs(got - float(want)) <= 4e-16 * float(want)
    assert sum(abs(a - b) for i, a in enumerate(BETA3) for b in BETA3[i + 1:]) == Fr(1295, 6)
    tau = float(wt.tau(wt.beta(q, 1)))
    assert abs(tau - float(TAU3)) <= 4e-16 * float(TAU3)
    # kappa of the first sub-stencil: 1 + (259/12)/(37/6) = 9/2
    assert 1 + TAU3 / BETA3[0] == Fr(9, 2)


G3 = mp.mpf(1) / (2 * mp.sqrt(3))      # Gauss nodes of m = 2 on [-1/2, 1/2]: -+G3
D1_3 = {"-1/2": (Fr(2, 3), Fr(1, 3)), "+1/2": (Fr(1, 3), Fr(2, 3)), "gauss": (Fr(1, 2), Fr(1, 2))}


@pytest.mark.parametrize("name,xi,eta,wx,wy,ax,ay,pt", [
    # EQP on the right x-edge at the upper Gauss node: (1/2, +G3), point index m + 1
    ("eqp", mp.mpf(1) / 2, G3, D1_3["+1/2"], D1_3["gauss"], 1, 3, 3),
    # CQP (-G3, +G3): h = 0, v = 1, point index 4m + v m + h
    ("cqp", -G3, G3, D1_3["gauss"], D1_3["gauss"], 2, 3, 10),
])
def test_weno3_value_worked_example(name, xi, eta, wx, wy, ax, ay, pt):
    """All linear weights are positive at every WENO3 point, so the split
    gives sigma+ = 2, sigma- = 1 and omega+ = omega-: the value is plain
    WENO-Z, sum omega_j p_j(xi, eta)."""
    gam = [wy[sy + 1] * wx[sx + 1] for sx, sy in SUBS3]
    pv = []
    for sx, sy in SUBS3:
        v00, b, c, d = bilinear3(sx, sy)
        pv.append(v00 + b * (xi - sx) + c * (eta - sy) + d * (xi - sx) * (eta - sy))
    want = wenoz_value(gam, BETA3, TAU3, pv)
    wt = WenoTables(3, 2, eps=0.0)
    q = torch.tensor(np.array(D3, dtype=np.float64))
    beta = wt.beta(q, 1)
    got = float(wt.value(q, 1, ax, ay, pt, beta, wt.tau(beta)))
    assert abs(got - float(want)) <= 1e-14 * abs(float(want)), (got, float(want))


# ----------------------------------------------------------------------------
# WENO5 worked example (n = 5, l = 3, s = 9): data a(x) + b(y)
# ----------------------------------------------------------------------------
AX = [0, 1, 3, 2, 7]      # a(x), x = -2..2
BY = [4, 0, 1, 5, 2]      # b(y), y = -2..2
STARTS5 = [-2, -1, 0]
SUBS5 = [(sx, sy) for sy in STARTS5 for sx in STARTS5]


def js5(f, s):
    """Jiang-Shu (1996) fifth-order smoothness indicator of the 3-cell
    sub-stencil starting at offset s (f indexed by offset + 2)."""
    g = lambda o: Fr(f[o + 2])
    if s == -2:
        return Fr(13, 12) * (g(-2) - 2 * g(-1) + g(0)) ** 2 + Fr(1, 4) * (g(-2) - 4 * g(-1) + 3 * g(0)) ** 2
    if s == -1:
        return Fr(13, 12) * (g(-1) - 2 * g(0) + g(1)) ** 2 + Fr(1, 4) * (g(-1) - g(1)) ** 2
    return Fr(13, 12) * (g(0) - 2 * g(1) + g(2)) ** 2 + Fr(1, 4) * (3 * g(0) - 4 * g(1) + g(2)) ** 2


def point5(f, s, where):
    """Textbook values of the quadratic from 3 cell averages at the right
    cell edge (x_{i+1/2}) and at the cell centre."""
    g = lambda o: Fr(f[o + 2])
    if where == "edge":
        return {-2: (2 * g(-2) - 7 * g(-1) + 11 * g(0)) / 6,
                -1: (-g(-1) + 5 * g(0) + 2 * g(1)) / 6,
                0: (2 * g(0) + 5 * g(1) - g(2)) / 6}[s]
    return {-2: (-g(-2) + 2 * g(-1) + 23 * g(0)) / 24,
            -1: (-g(-1) + 26 * g(0) - g(1)) / 24,
            0: (23 * g(0) + 2 * g(1) - g(2)) / 24}[s]


D1_5 = {"edge": (Fr(1, 10), Fr(6, 10), Fr(3, 10)), "centre": (Fr(-9, 80), Fr(49, 40), Fr(-9, 80))}


def _data5():
    return torch.tensor(np.array([[AX[x] + BY[y] for x in range(5)] for y in range(5)], dtype=np.float64))


def beta5_expected():
    return [js5(AX, sx) + js5(BY, sy) for sx, sy in SUBS5]


def tau5_expected():
    b = beta5_expected()
    return sum(abs(b[i] - b[j]) for i in range(9) for j in range(i + 1, 9)) * Fr(2, 90)


def test_weno5_beta_is_sum_of_jiang_shu_indicators():
    want = beta5_expected()
    # by hand, a: 13/12 + 75/4 = 22/3, 117/12 + 1/4 = 10, 39 + 16 = 55 for sx = -2, -1, 0;
    # b: 325/12 + 49/4 = 118/3, 117/12 + 25/4 = 16, 637/12 + 225/4 = 328/3 for sy = -2, -1, 0
    assert [js5(AX, s) for s in STARTS5] == [Fr(22, 3), Fr(10), Fr(55)]
    assert [js5(BY, s) for s in STARTS5] == [Fr(118, 3), Fr(16), Fr(328, 3)]
    wt = WenoTables(5, 3, eps=0.0)
    got = wt.beta(_data5(), 1).reshape(-1).tolist()
    for g, w in zip(got, want):
        assert abs(g - float(w)) <= 1e-15 * float(w)


def test_weno5_tau_worked_example():
    # the nine indicators are {22, 30, 165}/3 + {118, 48, 328}/3: 140, 148,
    # 283, 70, 78, 213, 350, 358, 493, all over 3; sorted, the 36 pair
    # differences add up to sum_k (2k - 8) x_k = 6174/3 = 2058, and
    # tau = 2/(9*10) * 2058 = 686/15
    xs = sorted(Fr(v, 3) for v in (140, 148, 283, 70, 78, 213, 350, 358, 493))
    assert sorted(beta5_expected()) == xs
    assert sum((2 * k - 8) * x for k, x in enumerate(xs)) == 2058
    assert tau5_expected() == Fr(686, 15)
    wt = WenoTables(5, 3, eps=0.0)
    got = float(wt.tau(wt.beta(_data5(), 1)))
    assert abs(got - float(tau5_expected())) <= 1e-15 * float(tau5_expected())


@pytest.mark.parametrize("name,wxk,wyk,ax,ay,pt", [
    # EQP on the right x-edge at the middle Gauss node (1/2, 0): point m + 1;
    # the y weights (-9/80, 49/40, -9/80) change sign, so the split matters
    ("eqp", "edge", "centre", 1, 3, 4),
    # CQP (0, 0): h = v = 1, point 4m + v m + h
    ("cqp", "centre", "centre", 3, 3, 16),
])
def test_weno5_split_value_worked_example(name, wxk, wyk, ax, ay, pt):
    wx, wy = D1_5[wxk], D1_5[wyk]
    gam = [wy[sy + 2] * wx[sx + 2] for sx, sy in SUBS5]
    assert any(g < 0 for g in gam)
    pv = [mp.mpf(point5(AX, sx, wxk).numerator) / point5(AX, sx, wxk).denominator
          + mp.mpf(point5(BY, sy, "centre").numerator) / point5(BY, sy, "centre").denominator for sx, sy in SUBS5]
    want = wenoz_value(gam, beta5_expected(), tau5_expected(), pv)
    wt = WenoTables(5, 3, eps=0.0)
    q = _data5()
    beta = wt.beta(q, 1)
    got = float(wt.value(q, 1, ax, ay, pt, beta, wt.tau(beta)))
    assert abs(got - float(want)) <= 1e-14 * abs(float(want)), (got, float(want))


def test_weno_epsilon_guards_a_flat_substencil():
    """(3.23) with epsilon = 1e-12: a flat sub-stencil (beta = 0) gets
    alpha = gamma (1 + tau/epsilon) and dominates the value, which is then
    its constant to within about epsilon/tau."""
    data = [row[:] for row in D3]
    data[0][0] = data[0][1] = data[1][0] = data[1][1] = 3          # sub-stencil (-1, -1) flat
    betas = []
    for sx, sy in SUBS3:
        v00 = data[sy + 1][sx + 1]
        b, c = data[sy + 1][sx + 2] - v00, data[sy + 2][sx + 1] - v00
        d = data[sy + 2][sx + 2] - data[sy + 1][sx + 2] - data[sy + 2][sx + 1] + v00
        betas.append(Fr(b - d * sy) ** 2 + Fr(c - d * sx) ** 2 + Fr(7, 6) * d * d)
    assert betas[0] == 0
    tau = sum(abs(betas[i] - betas[j]) for i in range(4) for j in range(i + 1, 4)) * Fr(1, 10)
    gam = [D1_3["gauss"][sy + 1] * D1_3["+1/2"][sx + 1] for sx, sy in SUBS3]
    xi, eta = mp.mpf(1) / 2, G3
    pv = []
    for sx, sy in SUBS3:
        v00 = data[sy + 1][sx + 1]
        b, c = data[sy + 1][sx + 2] - v00, data[sy + 2][sx + 1] - v00
        d = data[sy + 2][sx + 2] - data[sy + 1][sx + 2] - data[sy + 2][sx + 1] + v00
        pv.append(v00 + b * (xi - sx) + c * (eta - sy) + d * (xi - sx) * (eta - sy))
    eps = Fr(1, 10 ** 12)
    want = wenoz_value(gam, betas, tau, pv, eps=eps)
    wt = WenoTables(3, 2, eps=1e-12)
    q = torch.tensor(np.array(data, dtype=np.float64))
    beta = wt.beta(q, 1)
    got = float(wt.value(q, 1, 1, 3, 3, beta, wt.tau(beta)))
    assert abs(got - float(want)) <= 1e-14 * abs(float(want))
    assert abs(float(want) - 3.0) < 1e-11


# ----------------------------------------------------------------------------
# Planted slips: each must make one of the pins above fail
# ----------------------------------------------------------------------------
def _mutant(cls_or_fn, old, new):
    """A copy of an oracle function with one source fragment replaced."""
    src = textwrap.dedent(inspect.getsource(cls_or_fn))
    assert old in src, old
    src = src.replace(old, new, 1)
    lines = [ln for ln in src.splitlines() if not ln.lstrip().startswith("@")]
    ns = dict(vars(orhs))
    exec("\n".join(lines), ns)
    return ns[cls_or_fn.__name__]


WENO_SLIPS = [
    ("tau over ordered pairs", "tau", "for j in range(i + 1, s)", "for j in range(s)"),
    ("tau without 2/(s(s+1))", "tau", "t * (2.0 / (s * (s + 1)))", "t"),
    ("WENO-Z power 2", "value", "kappa = 1.0 + tau / (beta + self.eps)", "kappa = 1.0 + (tau / (beta + self.eps)) ** 2"),
    ("split sign", "value", "self.sp[pt] * (wp * ps).sum(0) - self.sm[pt]", "self.sp[pt] * (wp * ps).sum(0) + self.sm[pt]"),
    ("beta with transposed x/y", "beta", "Cf = torch.einsum(\"Bb,...ba,Aa->...BA\", My, cells, Mx)",
     "Cf = torch.einsum(\"Bb,...ba,Aa->...BA\", Mx, cells, My)"),
]


@pytest.mark.parametrize("label,fn,old,new", WENO_SLIPS, ids=[s[0] for s in WENO_SLIPS])
def test_weno_pins_catch_planted_slips(monkeypatch, label, fn, old, new):
    mut = _mutant(getattr(WenoTables, fn), old, new)
    monkeypatch.setattr(WenoTables, fn, staticmethod(mut) if fn == "tau" else mut)
    failed = 0
    for test in (test_weno3_value_worked_example, test_weno5_split_value_worked_example):
        for args in ([("eqp", mp.mpf(1) / 2, G3, D1_3["+1/2"], D1_3["gauss"], 1, 3, 3)]
                     if test is test_weno3_value_worked_example else
                     [("eqp", "edge", "centre", 1, 3, 4), ("cqp", "centre", "centre", 3, 3, 16)]):
            try:
                test(*args)
            except AssertionError:
                failed += 1
    assert failed >= 1, label


# ----------------------------------------------------------------------------
# LMARS (3.30)-(3.38) with jumps
# ----------------------------------------------------------------------------
def _state(X, Y, phi, u, v):
    sg = geo.sqrt_g(X, Y, A)
    return torch.tensor(np.stack([sg * phi, sg * phi * u, sg * phi * v]), dtype=torch.float64), sg


@pytest.mark.parametrize("direction", [1, 2])
@pytest.mark.parametrize("phiL,phiR", [(3.0e4, 2.0e4), (1.5e4, 2.6e4)])
def test_lmars_height_jump_at_rest(direction, phiL, phiR):
    """At rest on both sides: c = (sqrt(phiL) + sqrt(phiR))/2, so (3.32) gives
    m* = (phiL - phiR)/(2c) = sqrt(phiL) - sqrt(phiR) (flow from the deeper
    side), and (3.33) gives phi* = (phiL + phiR)/2.  The upwind mass flux is
    m sqrtG phi of the upwind side with m = m* sqrt(G^ii); the momentum flux
    is the pressure term (3.38) alone."""
    g = Grid(6, 3)
    X, Y = np.array([0.31]), np.array([-0.22])
    qL, sg = _state(X, Y, phiL, 0.0, 0.0)
    qR, _ = _state(X, Y, phiR, 0.0, 0.0)
    g11, g12, g22 = geo.g_upper(X, Y, A)
    gii = g11 if direction == 1 else g22
    mstar = math.sqrt(phiL) - math.sqrt(phiR)
    m = mstar * np.sqrt(gii)
    up = phiL if mstar > 0 else phiR
    pstar = 0.5 * (phiL + phiR)
    pres = 0.5 * sg * pstar ** 2
    want = np.stack([m * sg * up, pres * (g11 if direction == 1 else g12),
                     pres * (g12 if direction == 1 else g22)])
    got = g.lmars(qL, qR, X, Y, direction).numpy()
    assert np.allclose(got, want, rtol=1e-13, atol=0)


@pytest.mark.parametrize("direction", [1, 2])
def test_lmars_velocity_jump_equal_heights(direction):
    """Equal phi, normal velocities u_L > u_R (converging): c = sqrt(phi),
    m* = (uL_perp + uR_perp)/2 and phi* = phi + sqrt(phi)(uL_perp - uR_perp)/2,
    above phi (compression).  With m > 0 the flux is m q_L plus (3.38)."""
    g = Grid(6, 3)
    X, Y = np.array([-0.4]), np.array([0.17])
    phi = 2.2e4
    g11, g12, g22 = geo.g_upper(X, Y, A)
    gii = g11 if direction == 1 else g22
    unL, unR = 3.0e-6, 1.0e-6                  # contravariant normal components (rad/s)
    tang = 0.7e-6
    if direction == 1:
        qL, sg = _state(X, Y, phi, unL, tang)
        qR, _ = _state(X, Y, phi, unR, tang)
    else:
        qL, sg = _state(X, Y, phi, tang, unL)
        qR, _ = _state(X, Y, phi, tang, unR)
    pl, pr = unL / np.sqrt(gii), unR / np.sqrt(gii)
    mstar = 0.5 * (pl + pr)
    pstar = phi + math.sqrt(phi) * (pl - pr) / 2
    assert (pstar > phi).all()
    m = mstar * np.sqrt(gii)
    pres = 0.5 * sg * pstar ** 2
    P = np.stack([0 * pres, pres * (g11 if direction == 1 else g12), pres * (g12 if direction == 1 else g22)])
    want = m * qL.numpy() + P
    got = g.lmars(qL, qR, X, Y, direction).numpy()
    assert np.allclose(got, want, rtol=1e-13, atol=0)


def test_lmars_mirror_antisymmetry():
    """At X = 0 the metric is even in X (G^12 = 0).  Mirroring x -> -x swaps
    the sides and negates u: the mass and v-momentum fluxes change sign, the
    u-momentum flux does not."""
    g = Grid(6, 3)
    rng = np.random.default_rng(3)
    X, Y = np.zeros(20), rng.uniform(-0.9, 0.9, 20)
    phiL, phiR = rng.uniform(1e4, 3e4, 20), rng.uniform(1e4, 3e4, 20)
    uL, uR, vL, vR = (rng.uniform(-5e-6, 5e-6, 20) for _ in range(4))
    qL, _ = _state(X, Y, phiL, uL, vL)
    qR, _ = _state(X, Y, phiR, uR, vR)
    mL, _ = _state(X, Y, phiR, -uR, vR)
    mR, _ = _state(X, Y, phiL, -uL, vL)
    F = g.lmars(qL, qR, X, Y, 1).numpy()
    Fm = g.lmars(mL, mR, X, Y, 1).numpy()
    assert np.allclose(Fm, F * np.array([-1.0, 1.0, -1.0])[:, None], rtol=1e-12, atol=1e-12 * np.abs(F).max())


LMARS_SLIPS = [
    ("m* jump sign", "- (phiR - phiL) / c", "+ (phiR - phiL) / c"),
    ("phi* jump sign", "- c * (upR - upL)", "+ c * (upR - upL)"),
    ("upwind sign", "- mm.abs() * (qR - qL)", "+ mm.abs() * (qR - qL)"),
    ("m* half", "mstar = 0.5 * (upL + upR", "mstar = (upL + upR"),
]


@pytest.mark.parametrize("label,old,new", LMARS_SLIPS, ids=[s[0] for s in LMARS_SLIPS])
def test_lmars_pins_catch_planted_slips(monkeypatch, label, old, new):
    monkeypatch.setattr(Grid, "lmars", _mutant(Grid.lmars, old, new))
    failed = 0
    for fn, args in [(test_lmars_height_jump_at_rest, (1, 3.0e4, 2.0e4)),
                     (test_lmars_height_jump_at_rest, (2, 1.5e4, 2.6e4)),
                     (test_lmars_velocity_jump_equal_heights, (1,)),
                     (test_lmars_velocity_jump_equal_heights, (2,))]:
        try:
            fn(*args)
        except AssertionError:
            failed += 1
    assert failed >= 1, label
