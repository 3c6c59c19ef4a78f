"""Projection of the shared physical test fields onto the oracle's cell
averages.  Test infrastructure only.

A field f(p) -> (phi, us, vs) on unit vectors (see ``hope_inputs``) becomes
the state (sqrtG phi, sqrtG phi u, sqrtG phi v) of (2.15)-(2.16): the winds
are converted to contravariant components with the inverse of J (2.9)-(2.10)
and the cell average over dx dy is taken with an nq x nq Gauss rule.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import geometry as geo
from .weights import gauss


def cell_average(field, n: int, radius: float, nq: int = 8, pad: int = 0) -> torch.Tensor:
    """Cell averages (3, 6, n+2pad, n+2pad); with pad > 0 the outer cells are
    averages over each panel's extended coordinates (the exact ghost values)."""
    assert nq % 2 == 0, "an even rule keeps Gauss points off the panel centres"
    d = 0.5 * math.pi / n
    nodes, wts = gauss(nq)
    cen = geo.cell_centres(n, pad)
    xs = (cen[:, None] + nodes[None, :]) * d               # (n, nq)
    X = np.tan(xs)[None, None, :, :]                        # (1, 1, i, g)
    Y = np.tan(xs)[:, :, None, None]                        # (j, h, 1, 1)
    X, Y = np.broadcast_arrays(X, Y)                        # (j, h, i, g)
    w = (wts[None, :, None, None] * wts[None, None, None, :])
    out = np.zeros((3, 6, n + 2 * pad, n + 2 * pad))
    sg = geo.sqrt_g(X, Y, radius)
    for p in range(6):
        v = geo.panel_xyz(p, X, Y)
        phi, us, vs = field(v)
        lam, th = geo.lonlat(v)
        Ji = geo.inv2(geo.j_paper(p, lam, th, radius))
        u = Ji[0] * us + Ji[1] * vs
        vv = Ji[2] * us + Ji[3] * vs
        for c, val in enumerate((sg * phi, sg * phi * u, sg * phi * vv)):
            out[c, p] = (val * w).sum(axis=(1, 3))
    return torch.tensor(out)


def cell_sqrt_g(n: int, radius: float, nq: int = 8) -> np.ndarray:
    """Cell averages of sqrtG (n, n), identical on every panel."""
    d = 0.5 * math.pi / n
    nodes, wts = gauss(nq)
    xs = (geo.cell_centres(n, 0)[:, None] + nodes[None, :]) * d
    X = np.tan(xs)[None, None, :, :]
    Y = np.tan(xs)[:, :, None, None]
    w = wts[None, :, None, None] * wts[None, None, None, :]
    return (geo.sqrt_g(X, Y, radius) * w).sum(axis=(1, 3))
