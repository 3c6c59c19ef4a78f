"""Pins of the oracle's right-hand side (sections 2-3): conservation, design-order
convergence on exact steady states, WENO limits and bounds, LMARS consistency,
and the time schemes."""
import math

import numpy as np
import pytest
import torch

import hope_inputs as hi
from oracle import geometry as geo
from oracle.ic import cell_average
from oracle.norms import mass
from oracle.rhs import Grid, Params, WenoTables
from oracle.rk import ssp_rk3, ws_rk3

A = 6.371e6


def test_lmars_consistency_gives_physical_flux():
    """With q_L = q_R the LMARS flux is the exact flux F (x) or G (y) of (2.16)."""
    g = Grid(6, 3)
    rng = np.random.default_rng(0)
    X, Y = np.tan(rng.uniform(-0.78, 0.78, 50)), np.tan(rng.uniform(-0.78, 0.78, 50))
    sg = geo.sqrt_g(X, Y, A)
    g11, g12, g22 = geo.g_upper(X, Y, A)
    phi = rng.uniform(5e3, 3e4, 50)
    u, v = rng.uniform(-1e-5, 1e-5, 50), rng.uniform(-1e-5, 1e-5, 50)
    q = torch.tensor(np.stack([sg * phi, sg * phi * u, sg * phi * v]))
    F = g.lmars(q, q, X, Y, 1).numpy()
    Fx = np.stack([sg * phi * u, sg * (phi * u * u + 0.5 * g11 * phi ** 2), sg * (phi * u * v + 0.5 * g12 * phi ** 2)])
    Gf = g.lmars(q, q, X, Y, 2).numpy()
    Gy = np.stack([sg * phi * v, sg * (phi * u * v + 0.5 * g12 * phi ** 2), sg * (phi * v * v + 0.5 * g22 * phi ** 2)])
    assert np.allclose(F, Fx, rtol=1e-13, atol=0)
    assert np.allclose(Gf, Gy, rtol=1e-13, atol=0)


def test_lmars_upwinds():
    """Without a pressure jump the flux is m q_L for m > 0 and m q_R for m < 0."""
    g = Grid(6, 3)
    X, Y = np.array([0.1]), np.array([-0.2])
    sg = geo.sqrt_g(X, Y, A)
    phi = 2e4
    qL = torch.tensor(np.stack([sg * phi, sg * phi * 3e-6, sg * phi * 1e-6]))
    qR = torch.tensor(np.stack([sg * phi, sg * phi * 3e-6, sg * phi * -2e-6]))
    F = g.lmars(qL, qR, X, Y, 1)
    P = 0.5 * sg * phi ** 2 * np.array(geo.g_upper(X, Y, A))[[0, 0, 1]] * np.array([0, 1, 1])[:, None]
    assert torch.allclose(F - torch.tensor(P), 3e-6 * qL, rtol=1e-12)


@pytest.mark.parametrize("k,scheme", [(3, "tpp"), (5, "tpp"), (3, "weno"), (5, "weno"), (11, "tpp")])
def test_mass_conservation(k, scheme):
    """Total mass tendency vanishes to round-off (interior edges telescope; the
    two panels of a shared edge compute the same mass flux)."""
    n = 12 if k == 11 else 10
    g = Grid(n, k, scheme, Params(alpha=0.4))
    q = cell_average(hi.BalancedFlowWithCap(seed=3), n, A, nq=4)
    dq = g.tendency(q)
    d = 0.5 * math.pi / n
    scale = d * d * dq[0].abs().sum()
    assert abs(float(mass(dq))) < 2e-13 * float(scale)


@pytest.mark.parametrize("k,scheme,ns", [(3, "tpp", (12, 24)), (5, "tpp", (12, 24)), (5, "weno", (16, 32)),
                                         (7, "tpp", (16, 32))])
def test_balanced_flow_tendency_design_order(k, scheme, ns):
    """The exact steady state of (5.1)-(5.3) (tilted axis, tilted Coriolis):
    its discrete tendency is the truncation error, O(Delta^k) away from panel
    edges and O(Delta^(k-1)) next to them."""
    alpha = 0.7
    inner, full = [], []
    for n in ns:
        g = Grid(n, k, scheme, Params(alpha=alpha))
        q = cell_average(hi.BalancedFlow(alpha=alpha), n, A)
        rel = g.tendency(q).abs() / q.abs().amax((1, 2, 3), keepdim=True)
        a, b = n // 4, n - n // 4
        inner.append(float(rel[:, :, a:b, a:b].amax()))
        full.append(float(rel.amax()))
    assert math.log2(inner[0] / inner[1]) > k - 0.4
    assert math.log2(full[0] / full[1]) > k - 1.6


def test_lake_at_rest_tendency_vanishes_with_resolution():
    """A resting layer of constant depth is steady (d_j(sqrtG G^ij) = 0)."""
    vals = []
    for n in (10, 20):
        g = Grid(n, 5, "tpp")
        q = cell_average(hi.RestingLayer(seed=0, with_cap=False, pert=0.0), n, A)
        vals.append(float(g.tendency(q).abs().amax() / q[0].abs().max()))
    assert math.log2(vals[0] / vals[1]) > 3.5


def test_weno_linear_limit_is_tpp():
    """With the nonlinear weights switched off (epsilon -> infinity, so
    omega+- = gamma+-/sigma+-) genuine 2D WENO-n is exactly TPP-n."""
    n = 8
    q = cell_average(hi.BalancedFlowWithCap(seed=5), n, A, nq=4)
    w = Grid(n, 5, "weno", Params(alpha=0.3, weno_eps=1e300)).tendency(q)
    t = Grid(n, 5, "tpp", Params(alpha=0.3)).tendency(q)
    for v in range(3):
        assert float((w[v] - t[v]).abs().max() / t[v].abs().max()) < 1e-11


def _poly_averages(f_int, size):
    """Cell averages on a size x size unit grid centred on the target cell of
    the polynomial with antiderivative pair f_int (exact for polynomials)."""
    c = size // 2
    out = np.zeros((size, size))
    for j in range(size):
        for i in range(size):
            out[j, i] = f_int(i - c - 0.5, i - c + 0.5, j - c - 0.5, j - c + 0.5)
    return torch.tensor(out)


@pytest.mark.parametrize("name,fint,beta", [
    ("x", lambda a, b, c, d: (b * b - a * a) / 2 * (d - c), 1.0),
    ("x^2", lambda a, b, c, d: (b ** 3 - a ** 3) / 3 * (d - c), 13.0 / 3.0),
    ("xy", lambda a, b, c, d: (b * b - a * a) / 2 * (d * d - c * c) / 2, 7.0 / 6.0),
    ("1", lambda a, b, c, d: (b - a) * (d - c), 0.0),
])
def test_smoothness_indicator_closed_forms(name, fint, beta):
    """beta = sum over (a,b) != (0,0) of the integral of (d^a_x d^b_y p)^2 over
    the unit target cell: x -> 1, x^2 -> 1/3 + 4, xy -> 1/12 + 1/12 + 1."""
    wt = WenoTables(5, 3)
    qpad = _poly_averages(fint, 5)
    b = wt.beta(qpad, 1)
    assert np.allclose(b.numpy().ravel(), beta, atol=1e-13)


def test_weno_reproduces_low_degree_polynomials():
    """Data from a polynomial of degree < l in each variable is reproduced
    exactly at every point whatever the nonlinear weights are."""
    wt = WenoTables(5, 3)
    f = lambda a, b, c, d: ((b ** 3 - a ** 3) / 3 + 2 * (b * b - a * a) / 2) * ((d * d - c * c) / 2 + (d - c))
    qpad = _poly_averages(f, 5)
    beta = wt.beta(qpad, 1)
    tau = wt.tau(beta)
    from oracle.weights import cell_points
    pts = cell_points(3)
    for pt, (x, y) in enumerate(pts):
        ax = {-0.5: 0, 0.5: 1}.get(round(x, 12), None)
        ay = {-0.5: 0, 0.5: 1}.get(round(y, 12), None)
        nodes = [-0.3872983346207417, 0.0, 0.3872983346207417]
        ax = ax if ax is not None else 2 + int(np.argmin([abs(x - t) for t in nodes]))
        ay = ay if ay is not None else 2 + int(np.argmin([abs(y - t) for t in nodes]))
        val = float(wt.value(qpad, 1, ax, ay, pt, beta, tau))
        assert abs(val - (x ** 2 + 2 * x) * (y + 1)) < 1e-13


def test_weno_bounded_across_a_step():
    """Across a jump the reconstructed edge values stay within the data range
    (to within a small fraction of the jump), where TPP-5 overshoots."""
    wt = WenoTables(5, 3)
    data = np.ones((5, 5))
    data[:, 3:] = 2.0                      # jump between the target cell and its right neighbour
    qpad = torch.tensor(data)
    beta = wt.beta(qpad, 1)
    tau = wt.tau(beta)
    from oracle.weights import axis_weights, centred
    for h in range(3):
        val = float(wt.value(qpad, 1, 1, 2 + h, 3 + h, beta, tau))     # right edge
        assert 1.0 - 1e-6 <= val <= 1.0 + 0.05
    wc = axis_weights(centred(5), 3)
    tpp = float(sum(wc[2 + 1][b] * wc[1][a] * data[b, a] for b in range(5) for a in range(5)))
    assert tpp > 1.3


def test_rk_stability_polynomials():
    """Both three-stage schemes have amplification 1 + z + z^2/2 + z^3/6."""
    for z in (-0.5, 0.3, -2.0 + 0.5j):
        lam = complex(z)
        L = lambda y: lam * y
        expect = 1 + lam + lam ** 2 / 2 + lam ** 3 / 6
        assert abs(ssp_rk3(L, 1.0 + 0j, 1.0) - expect) < 1e-14
        assert abs(ws_rk3(L, 1.0 + 0j, 1.0) - expect) < 1e-14
