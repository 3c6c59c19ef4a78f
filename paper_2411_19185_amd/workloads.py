"""Synthetic benchmark states: the shared seeded physical fields (hope_inputs)
projected onto this library's cell averages.

Input preparation only (not part of the right-hand side): each cell average
of q = (sqrtG phi, sqrtG phi u, sqrtG phi v) is an nq x nq Gauss average of
the pointwise field, with the winds converted to contravariant components
through the covariant basis of the panel map.  Uses numpy on the host.
"""
from __future__ import annotations

import math

import numpy as np

import hope_inputs as hi

# unnormalised direction of (X, Y) on each panel, as (const, X, Y) coefficient
# rows for the three Cartesian components
_MAP = np.array([
    [[1, 0, 0], [0, 1, 0], [0, 0, 1]],
    [[0, -1, 0], [1, 0, 0], [0, 0, 1]],
    [[-1, 0, 0], [0, -1, 0], [0, 0, 1]],
    [[0, 1, 0], [-1, 0, 0], [0, 0, 1]],
    [[0, 0, -1], [0, 1, 0], [1, 0, 0]],
    [[0, 0, 1], [0, 1, 0], [-1, 0, 0]],
], dtype=np.float64)


def _panel_points(p, X, Y, radius):
    c = _MAP[p]
    v = np.stack([c[i, 0] + c[i, 1] * X + c[i, 2] * Y for i in range(3)], -1)
    dX = np.broadcast_to(c[:, 1], v.shape)
    dY = np.broadcast_to(c[:, 2], v.shape)
    d2 = (v * v).sum(-1, keepdims=True)
    d = np.sqrt(d2)
    u = v / d
    ex = radius * (1 + X * X)[..., None] * (dX / d - v * (v * dX).sum(-1, keepdims=True) / (d * d2))
    ey = radius * (1 + Y * Y)[..., None] * (dY / d - v * (v * dY).sum(-1, keepdims=True) / (d * d2))
    return u, ex, ey


def cell_average(field, n: int, radius: float = hi.EARTH_RADIUS, nq: int = 2) -> np.ndarray:
    """(3, 6, n, n) cell averages of the state for the field f(p) -> (phi, us, vs)."""
    x0, w0 = np.polynomial.legendre.leggauss(nq)
    nodes, wts = x0 / 2, w0 / 2
    d = 0.5 * math.pi / n
    xs = ((np.arange(n) + 0.5 - n / 2.0)[:, None] + nodes[None, :]) * d          # (n, nq)
    X = np.broadcast_to(np.tan(xs)[None, None, :, :], (n, nq, n, nq))           # (j, h, i, g)
    Y = np.broadcast_to(np.tan(xs)[:, :, None, None], (n, nq, n, nq))
    w = wts[None, :, None, None] * wts[None, None, None, :]
    out = np.zeros((3, 6, n, n))
    for p in range(6):
        u, ex, ey = _panel_points(p, X, Y, radius)
        g11 = (ex * ex).sum(-1)
        g12 = (ex * ey).sum(-1)
        g22 = (ey * ey).sum(-1)
        det = g11 * g22 - g12 * g12
        sg = np.sqrt(det)
        phi, us, vs = field(u)
        lam = np.arctan2(u[..., 1], u[..., 0])
        sth = u[..., 2]
        cth = np.sqrt(np.maximum(0.0, 1 - sth * sth))
        east = np.stack([-np.sin(lam), np.cos(lam), np.zeros_like(lam)], -1)
        north = np.stack([-sth * np.cos(lam), -sth * np.sin(lam), cth], -1)
        V = us[..., None] * east + vs[..., None] * north
        b1 = (ex * V).sum(-1)
        b2 = (ey * V).sum(-1)
        uc = (g22 * b1 - g12 * b2) / det
        vc = (-g12 * b1 + g11 * b2) / det
        for c, val in enumerate((sg * phi, sg * phi * uc, sg * phi * vc)):
            out[c, p] = (val * w).sum(axis=(1, 3))
    return out


def smooth_random_state(n: int, seed: int, nq: int = 2) -> np.ndarray:
    """Resting 1000 m layer plus a 1 % seeded spherical-harmonic perturbation."""
    return cell_average(hi.RestingLayer(seed=seed, with_cap=False), n, nq=nq)


def dam_break_state(n: int, seed: int, nq: int = 2) -> np.ndarray:
    return cell_average(hi.RestingLayer(seed=seed), n, nq=nq)


def member_state(n: int, seed: int, nq: int = 2):
    f = hi.BalancedFlowWithCap(seed=seed)
    return f.alpha, cell_average(f, n, nq=nq)


def cell_sqrt_g(n: int, radius: float = hi.EARTH_RADIUS, nq: int = 4) -> np.ndarray:
    """(n, n) cell averages over dx dy of sqrtG = a^2 (1+X^2)(1+Y^2) / (1+X^2+Y^2)^(3/2)
    (the same on every panel); converts a mass cell average to a height."""
    x0, w0 = np.polynomial.legendre.leggauss(nq)
    d = 0.5 * math.pi / n
    xs = ((np.arange(n) + 0.5 - n / 2.0)[:, None] + x0[None, :] / 2) * d
    X = np.tan(xs)[None, None, :, :]
    Y = np.tan(xs)[:, :, None, None]
    sg = radius ** 2 * (1 + X * X) * (1 + Y * Y) / (1 + X * X + Y * Y) ** 1.5
    w = (w0[None, :, None, None] / 2) * (w0[None, None, None, :] / 2)
    return (sg * w).sum(axis=(1, 3))


def cfl_dt(q: np.ndarray, radius: float = hi.EARTH_RADIUS, cfl: float = 0.5) -> float:
    """Time step for a given Courant number from the largest gravity-wave plus
    advection speed of the state (dt is an input of the method)."""
    n = q.shape[-1]
    d = 0.5 * math.pi / n
    x = (np.arange(n) + 0.5 - n / 2) * d
    X = np.tan(x)[None, :]
    Y = np.tan(x)[:, None]
    d2 = 1 + X * X + Y * Y
    sg = radius ** 2 * (1 + X * X) * (1 + Y * Y) / d2 ** 1.5
    phi = q[0] / sg
    u = q[1] / q[0]
    v = q[2] / q[0]
    g11 = d2 / (radius ** 2 * (1 + X * X))
    g22 = d2 / (radius ** 2 * (1 + Y * Y))
    s = np.maximum(np.abs(u) + np.sqrt(phi * g11), np.abs(v) + np.sqrt(phi * g22))
    return cfl * d / float(s.max())
