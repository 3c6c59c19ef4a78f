"""Cubed-sphere geometry for the oracle (section 2).  Test infrastructure only.

Panels are numbered 0..5 here (the paper's 1..6, Figure 2.1): 0-3 around
the equator, 4 north, 5 south.  On each panel the equiangular coordinates
(x, y) lie in [-pi/4, pi/4], X = tan x, Y = tan y, delta^2 = 1 + X^2 + Y^2.

The panel maps are not printed in the paper; they are the gnomonic maps that
satisfy the printed latitude relation (2.5) and whose derivatives reproduce
the printed conversion matrix J (2.10)-(2.11) (both checked by the tests):

  panel 0: (1, X, Y)/delta     panel 1: (-X, 1, Y)/delta
  panel 2: (-1, -X, Y)/delta   panel 3: (X, -1, Y)/delta
  panel 4: (-Y, X, 1)/delta    panel 5: (Y, X, -1)/delta

The same formulas define each panel's extended coordinates beyond its edges
(used for ghost cells).
"""
from __future__ import annotations

import math

import numpy as np

PANEL_AXIS = np.array([[1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], dtype=np.float64)


def panel_xyz(p: int, X, Y):
    """Unit vector of the point (X, Y) of panel p (extended coordinates allowed)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    one = np.ones_like(X + Y)
    X = X * one
    Y = Y * one
    comps = {
        0: (one, X, Y),
        1: (-X, one, Y),
        2: (-one, -X, Y),
        3: (X, -one, Y),
        4: (-Y, X, one),
        5: (Y, X, -one),
    }[p]
    v = np.stack(comps, axis=-1)
    return v / np.sqrt(1.0 + X * X + Y * Y)[..., None]


def xyz_to_XY(p: int, v):
    """Inverse of panel_xyz: the (X, Y) of direction v in panel p's coordinates."""
    a, b, c = v[..., 0], v[..., 1], v[..., 2]
    if p == 0:
        return b / a, c / a
    if p == 1:
        return -a / b, c / b
    if p == 2:
        return b / a, -c / a
    if p == 3:
        return -a / b, -c / b
    if p == 4:
        return b / c, -a / c
    return -b / c, -a / c


def signed_components(v):
    """(..., 6) components of v along the six panel axes."""
    return v @ PANEL_AXIS.T


def owners(v, rtol=1e-12):
    """Owner panel(s) of direction v: the panel whose axis has the largest
    component.  Returns (best, second, tie) where tie marks points whose two
    largest components agree to rtol (the diagonals of corner ghost blocks)."""
    s = signed_components(v)
    order = np.argsort(-s, axis=-1, kind="stable")
    best = order[..., 0]
    second = order[..., 1]
    sb = np.take_along_axis(s, best[..., None], -1)[..., 0]
    ss = np.take_along_axis(s, second[..., None], -1)[..., 0]
    tie = np.abs(sb - ss) <= rtol * np.abs(sb)
    return best, second, tie


def lonlat(v):
    lam = np.arctan2(v[..., 1], v[..., 0])
    th = np.arcsin(np.clip(v[..., 2], -1.0, 1.0))
    return lam, th


# ----------------------------------------------------------------------------
# Metric, (2.6)-(2.8), written literally
# ----------------------------------------------------------------------------
def sqrt_g(X, Y, a):
    """(2.8): sqrt(G) = a^2 (1+X^2)(1+Y^2) / delta^3."""
    d = np.sqrt(1.0 + X * X + Y * Y)
    return a * a * (1.0 + X * X) * (1.0 + Y * Y) / d ** 3


def g_upper(X, Y, a):
    """(2.6), with the denominator (1+X^2)(1+Y^2): returns G^11, G^12, G^22."""
    d2 = 1.0 + X * X + Y * Y
    s = d2 / (a * a * (1.0 + X * X) * (1.0 + Y * Y))
    return s * (1.0 + Y * Y), s * X * Y, s * (1.0 + X * X)


def g_lower(X, Y, a):
    """(2.7): returns G_11, G_12, G_22."""
    d2 = 1.0 + X * X + Y * Y
    s = a * a * (1.0 + X * X) * (1.0 + Y * Y) / (d2 * d2)
    return s * (1.0 + X * X), -s * X * Y, s * (1.0 + Y * Y)


def j_paper(p: int, lam, th, a):
    """The wind conversion matrix J of (2.10)-(2.11) for panel p (0-based),
    as printed: (us, vs) = J (u, v).  Returns (J11, J12, J21, J22)."""
    if p < 4:
        lp = lam - 0.5 * math.pi * p
        ct, st = np.cos(th), np.sin(th)
        return (a * ct, np.zeros_like(ct),
                -a * st * ct * np.tan(lp),
                a * (np.cos(lp) * ct * ct + st * st / np.cos(lp)))
    st = np.sin(th)
    tt = np.tan(th)
    g1 = 1.0 + np.sin(lam) ** 2 / tt ** 2
    g2 = 1.0 + np.cos(lam) ** 2 / tt ** 2
    if p == 4:
        return (a * np.cos(lam) * st * g1, a * np.sin(lam) * st * g2,
                -a * np.sin(lam) * st * st * g1, a * np.cos(lam) * st * st * g2)
    return (-a * np.cos(lam) * st * g1, a * np.sin(lam) * st * g2,
            a * np.sin(lam) * st * st * g1, a * np.cos(lam) * st * st * g2)


def inv2(m):
    a, b, c, d = m
    det = a * d - b * c
    return d / det, -b / det, -c / det, a / det


def mul2(m, n):
    a, b, c, d = m
    e, f, g, h = n
    return a * e + b * g, a * f + b * h, c * e + d * g, c * f + d * h


def coriolis_f(v, omega, alpha):
    """f = 2 Omega sin(theta') with the rotation axis tilted by alpha towards
    -x; with alpha = 0 this is 2 Omega sin(theta) of (2.3)-(2.5)."""
    return 2.0 * omega * (-math.sin(alpha) * v[..., 0] + math.cos(alpha) * v[..., 2])


def cell_centres(n: int, r: int):
    """Centres, in units of Delta, of cells -r..n+r-1 (exactly antisymmetric)."""
    i = np.arange(-r, n + r)
    return (i + 0.5 - n / 2.0)
