"""Pins of the oracle's cubed-sphere geometry against section 2."""
import math

import numpy as np
import pytest

from oracle import geometry as geo
from oracle.ic import cell_sqrt_g

A = 6.371e6


def _rand(p, n=200, lim=0.78):
    rng = np.random.default_rng(p)
    return rng.uniform(-lim, lim, n), rng.uniform(-lim, lim, n)


@pytest.mark.parametrize("p", range(6))
def test_latitude_relation_2_5(p):
    x, y = _rand(p)
    X, Y = np.tan(x), np.tan(y)
    d = np.sqrt(1 + X * X + Y * Y)
    st = geo.panel_xyz(p, X, Y)[..., 2]
    expect = Y / d if p < 4 else (1 / d if p == 4 else -1 / d)
    assert np.abs(st - expect).max() < 1e-15


@pytest.mark.parametrize("p", range(6))
def test_map_derivative_matches_printed_J(p):
    """Finite differences of (lambda, theta) along the panel map reproduce the
    printed conversion matrix (2.10)-(2.11), which fixes the orientation of
    every panel's coordinates."""
    x, y = _rand(p, lim=0.7)
    h = 1e-6

    def ll(x, y):
        return geo.lonlat(geo.panel_xyz(p, np.tan(x), np.tan(y)))

    wrap = lambda d: (d + np.pi) % (2 * np.pi) - np.pi
    l0, t0 = ll(x, y)
    lxp, txp = ll(x + h, y)
    lxm, txm = ll(x - h, y)
    lyp, typ = ll(x, y + h)
    lym, tym = ll(x, y - h)
    Jfd = (A * np.cos(t0) * wrap(lxp - lxm) / (2 * h), A * np.cos(t0) * wrap(lyp - lym) / (2 * h),
           A * (txp - txm) / (2 * h), A * (typ - tym) / (2 * h))
    Jp = geo.j_paper(p, l0, t0, A)
    for u, w in zip(Jfd, Jp):
        assert np.abs(u - w).max() < 1e-8 * A


@pytest.mark.parametrize("p", range(6))
def test_metric_identities(p):
    """(2.12) J^T J = G_ij; (2.6) (denominator (1+X^2)(1+Y^2)) inverts (2.7);
    (2.8) sqrtG^2 = det G_ij."""
    x, y = _rand(p, lim=0.7)
    X, Y = np.tan(x), np.tan(y)
    lam, th = geo.lonlat(geo.panel_xyz(p, X, Y))
    J = geo.j_paper(p, lam, th, A)
    G11, G12, G22 = geo.g_lower(X, Y, A)
    JtJ = (J[0] ** 2 + J[2] ** 2, J[0] * J[1] + J[2] * J[3], J[1] ** 2 + J[3] ** 2)
    for u, w in zip(JtJ, (G11, G12, G22)):
        assert np.abs(u - w).max() < 1e-14 * np.abs(G11).max()
    g11, g12, g22 = geo.g_upper(X, Y, A)
    assert np.allclose(g11 * G11 + g12 * G12, 1, atol=1e-14)
    assert np.allclose(g11 * G12 + g12 * G22, 0, atol=1e-14)
    assert np.allclose(g12 * G12 + g22 * G22, 1, atol=1e-14)
    sg = geo.sqrt_g(X, Y, A)
    assert np.allclose(sg ** 2, G11 * G22 - G12 ** 2, rtol=1e-14)


def test_pressure_metric_identity():
    """d/dx (sqrtG G^11) + d/dy (sqrtG G^12) = 0 (so a lake at rest is steady)."""
    x, y = _rand(7, lim=0.7)
    h = 1e-5

    def f(x, y, comp):
        X, Y = np.tan(x), np.tan(y)
        g = geo.g_upper(X, Y, A)
        return geo.sqrt_g(X, Y, A) * g[comp]

    div1 = (f(x + h, y, 0) - f(x - h, y, 0)) / (2 * h) + (f(x, y + h, 1) - f(x, y - h, 1)) / (2 * h)
    div2 = (f(x + h, y, 1) - f(x - h, y, 1)) / (2 * h) + (f(x, y + h, 2) - f(x, y - h, 2)) / (2 * h)
    assert np.abs(div1).max() < 1e-8 and np.abs(div2).max() < 1e-8


def test_sphere_area():
    n = 24
    d = 0.5 * math.pi / n
    total = 6 * cell_sqrt_g(n, A).sum() * d * d
    assert abs(total - 4 * math.pi * A * A) < 1e-12 * 4 * math.pi * A * A


@pytest.mark.parametrize("p", range(6))
def test_inverse_map_and_owner(p):
    x, y = _rand(p)
    X, Y = np.tan(x), np.tan(y)
    v = geo.panel_xyz(p, X, Y)
    Xb, Yb = geo.xyz_to_XY(p, v)
    assert np.allclose(Xb, X, atol=1e-14) and np.allclose(Yb, Y, atol=1e-14)
    best, _, _ = geo.owners(v)
    assert (best == p).all()


def test_coriolis_untilted_is_2_omega_sin_theta():
    v = geo.panel_xyz(0, np.tan(0.3), np.tan(-0.2))
    f = geo.coriolis_f(v, 7.292e-5, 0.0)
    assert abs(f - 2 * 7.292e-5 * v[2]) < 1e-20
