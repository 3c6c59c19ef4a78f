"""Pins of the oracle's bottom topography (section 2, (2.13)-(2.14)): the
reconstruction of sqrtG phi_t, the pressure with phi_t, and the source psi_B.

  * the closed form of d(ln sqrtG)/dx against finite differences of (2.8);
  * the derivative weights reproduce derivatives of polynomials exactly;
  * a zero surface gives exactly the tendency without topography;
  * the "C-property" the reformulation is for: a lake at rest with a flat
    free surface over the section 5.2 cone (5.8), whose slope jumps at the
    peak and along the rim, has the residual tendency of the same lake over
    a flat bottom (the metric truncation of sqrtG phi_t, which converges at
    order k - 1 in the maximum norm), not one set by the mountain's kinks;
  * an exact steady state with topography (the tilted balanced flow over a
    ridge that is constant along its flow lines): its discrete tendency is
    the truncation error.  psi_B takes d(phi_t)/dx^j from the derivative of
    the order-k polynomial, which is accurate to order k - 1, so the residual
    converges at order k - 1 or better (measured: k - 0.9 to k - 0.4);
  * mass is conserved to round-off over the mountain;
and planted slips (pressure without phi_s, psi_B dropped or with the wrong
sign, the wrong metric derivative) make these fail."""
import inspect
import math
import textwrap

import numpy as np
import pytest
import torch

import hope_inputs as hi
import oracle.rhs as orhs
from oracle import geometry as geo
from oracle import weights as W
from oracle.ic import cell_average
from oracle.norms import mass
from oracle.rhs import Grid, Params

A = hi.EARTH_RADIUS


def test_log_sqrt_g_derivative_closed_form():
    """d(ln sqrtG)/dx = X (2Y^2 - X^2 - 1)/delta^2 with X = tan x, from (2.8)."""
    rng = np.random.default_rng(5)
    x, y = rng.uniform(-0.9, 0.9, 40), rng.uniform(-0.9, 0.9, 40)
    h = 1e-6
    fd = (np.log(geo.sqrt_g(np.tan(x + h), np.tan(y), A)) - np.log(geo.sqrt_g(np.tan(x - h), np.tan(y), A))) / (2 * h)
    X, Y = np.tan(x), np.tan(y)
    closed = X * (2 * Y * Y - X * X - 1) / (1 + X * X + Y * Y)
    assert np.abs(fd - closed).max() < 1e-8


@pytest.mark.parametrize("k", [3, 5, 7, 11])
def test_derivative_weights_reproduce_polynomial_derivatives(k):
    """From the cell averages of x^j (j < k) the derivative weights give
    j xi^(j-1) at every axis point, exactly up to rounding."""
    m = (k + 1) // 2
    offs = W.centred(k)
    wd = W.axis_derivative_weights(offs, m)
    pts = [float(v) for v in W.edge_points_mp(m)]
    for j in range(k):
        avg = np.array([float(W.cell_moment(o, j)) for o in offs])
        for a, xi in enumerate(pts):
            want = j * xi ** (j - 1) if j else 0.0
            assert abs(wd[a] @ avg - want) < 1e-14 * (np.abs(wd[a] * avg).sum() + 1.0)


@pytest.mark.parametrize("k,scheme", [(3, "tpp"), (5, "weno")])
def test_zero_surface_is_the_flat_bottom(k, scheme):
    n = 8
    q = cell_average(hi.BalancedFlowWithCap(seed=3), n, A, nq=4)
    flat = Grid(n, k, scheme, Params(alpha=0.4)).tendency(q)
    zero = Grid(n, k, scheme, Params(alpha=0.4, surface=lambda p: np.zeros(p.shape[:-1]))).tendency(q)
    assert torch.equal(flat, zero)


def _lake_rates(k, scheme, ns, surface):
    vals = []
    for n in ns:
        g = Grid(n, k, scheme, Params(surface=surface))
        flat = lambda p: np.zeros(p.shape[:-1])
        q = cell_average(hi.LakeAtRest(surface=surface or flat), n, A, nq=4)
        vals.append(float(g.tendency(q).abs().amax() / q[0].abs().max()))
    return vals


@pytest.mark.parametrize("k,scheme,ns", [(3, "tpp", (12, 24)), (5, "tpp", (12, 24)), (5, "weno", (16, 32))])
def test_lake_at_rest_over_the_cone_keeps_design_order(k, scheme, ns):
    """C-property: the reconstruction variable sqrtG phi_t of a flat free
    surface is the same with and without the mountain, so the residual over
    the kinked cone is the flat-bottom lake's, and vanishes as fast."""
    over = _lake_rates(k, scheme, ns, hi.ConeMountain())
    flat = _lake_rates(k, scheme, ns, None)
    assert math.log2(over[0] / over[1]) > k - 1.4, over
    assert all(o <= 1.05 * f for o, f in zip(over, flat)), (over, flat)


@pytest.mark.parametrize("k,scheme,ns", [(3, "tpp", (12, 24)), (5, "tpp", (12, 24)), (5, "weno", (16, 32))])
def test_steady_flow_over_a_ridge_converges_at_design_order(k, scheme, ns):
    alpha = 0.7
    inner, full = [], []
    for n in ns:
        f = hi.BalancedFlowOverRidge(alpha=alpha)
        g = Grid(n, k, scheme, Params(alpha=alpha, surface=f.surface))
        q = cell_average(f, n, A)
        rel = g.tendency(q).abs() / q.abs().amax((1, 2, 3), keepdim=True)
        a, b = n // 4, n - n // 4
        inner.append(float(rel[:, :, a:b, a:b].amax()))
        full.append(float(rel.amax()))
    assert math.log2(inner[0] / inner[1]) > k - 1.3, inner
    assert math.log2(full[0] / full[1]) > k - 1.6, full


@pytest.mark.parametrize("k,scheme", [(3, "weno"), (5, "tpp")])
def test_mass_conservation_over_the_mountain(k, scheme):
    n = 10
    f = hi.MountainFlow(radius=A)
    g = Grid(n, k, scheme, Params(surface=f.surface))
    q = cell_average(f, n, A, nq=4)
    dq = g.tendency(q)
    d = 0.5 * math.pi / n
    assert abs(float(mass(dq))) < 2e-13 * float(d * d * dq[0].abs().sum())


def _mutant(fn, old, new):
    src = textwrap.dedent(inspect.getsource(fn))
    assert old in src, old
    src = src.replace(old, new, 1)
    ns = dict(vars(orhs))
    exec(src, ns)
    return ns[fn.__name__]


SLIPS = [
    ("pressure without phi_s", "lmars", "phistar = phistar + phis", "phistar = phistar"),
    ("psi_B dropped", "sources", "Sbar1 + w * (psiM1 + psiC1 + psiB1)", "Sbar1 + w * (psiM1 + psiC1)"),
    ("psi_B sign", "sources", "psiB1 = sp * (g11 * dx + g12 * dy)", "psiB1 = -sp * (g11 * dx + g12 * dy)"),
    ("metric derivative sign", "sources", "dx = (Txi / self.delta - Tt", "dx = (Txi / self.delta + Tt"),
]


@pytest.mark.parametrize("label,fn,old,new", SLIPS, ids=[s[0] for s in SLIPS])
def test_topography_pins_catch_planted_slips(monkeypatch, label, fn, old, new):
    monkeypatch.setattr(Grid, fn, _mutant(getattr(Grid, fn), old, new))
    failed = 0
    for test, args in [(test_lake_at_rest_over_the_cone_keeps_design_order, (5, "tpp", (12, 24))),
                       (test_steady_flow_over_a_ridge_converges_at_design_order, (5, "tpp", (12, 24)))]:
        try:
            test(*args)
        except AssertionError:
            failed += 1
    assert failed >= 1, label
