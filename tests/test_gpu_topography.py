"""GPU parity of the bottom topography (section 2, (2.13)-(2.14)): the HIP
path through the C ABI, with the surface geopotential passed as a host
callback, against the oracle on the same seeded fields, at 1e-11 relative
(L-infinity over all cells, per variable).

States, each times (1 + 1 % seeded smooth random field) so that it is not in
balance: the flow over the isolated cone mountain of section 5.2 (5.8), the
steady flow over a ridge about the tilted rotation axis, and the lake at rest
over the cone (compared after two Runge-Kutta steps).  The balanced states
themselves are ill-conditioned for a tendency comparison: their tendency is
the truncation error left after O(1) terms cancel, and moving the oracle's
own input by 1e-15 moves it by up to 3e-8 (ridge, TPP9); the perturbed
states move it by about 1e-12.  Also the C-property on the GPU path itself,
a five-day run of the section 5.2 case, and the refusal of a surface that is
not finite."""
import math

import numpy as np
import pytest
import torch

import hope_inputs as hi
from cases import cfl_dt, rel_err, smooth_cell_field, to_padded
from oracle.ic import cell_average
from oracle.rhs import Grid as OracleGrid
from oracle.rhs import Params
from oracle.rk import ssp_rk3

pytestmark = pytest.mark.gpu

TOL = 1e-11
A = hi.EARTH_RADIUS


def _field(name, seed):
    if name == "mountain":
        f = hi.MountainFlow(radius=A)
        return 0.0, f, f.surface
    if name == "ridge":
        alpha = hi.draw_tilt(seed)
        f = hi.BalancedFlowOverRidge(alpha=alpha)
        return alpha, f, f.surface
    cone = hi.ConeMountain()
    return 0.0, hi.LakeAtRest(surface=cone), cone


def _state(name, n, seed):
    alpha, f, surface = _field(name, seed)
    q = cell_average(f, n, A, nq=4)
    return alpha, q * (1.0 + 1e-2 * smooth_cell_field(n, seed + 4000)), surface


def _grids(n, order, scheme, alpha, surface):
    from paper_2411_19185_amd import Grid
    og = OracleGrid(n, order, scheme, Params(alpha=alpha, surface=surface))
    return og, Grid(n, order, scheme, axis_tilt=alpha, surface=surface)


CASES = [
    # (n, order, scheme, state, seed)
    (24, 3, "tpp", "mountain", 0),
    (16, 5, "tpp", "mountain", 0),
    (20, 5, "weno", "mountain", 0),
    (13, 3, "weno", "mountain", 0),        # ragged: odd n
    (18, 7, "tpp", "mountain", 0),
    (12, 11, "tpp", "mountain", 0),        # cell nodes in chunks
    (45, 5, "weno", "mountain", 0),        # full strips of 45 columns
    (20, 5, "weno", "ridge", 3),
    (16, 9, "tpp", "ridge", 4),
]


@pytest.mark.parametrize("n,order,scheme,state,seed", CASES)
def test_tendency_with_topography_matches_oracle(n, order, scheme, state, seed):
    print(f"case n={n} order={order} {scheme} {state} (perturbed) seed={seed}", flush=True)
    alpha, q, surface = _state(state, n, seed)
    og, g = _grids(n, order, scheme, alpha, surface)
    ref = og.tendency(q)
    out = g.tendency(to_padded(q, g.r))
    torch.cuda.synchronize()
    err = rel_err(out, ref)
    print("rel err", err, flush=True)
    assert max(err) < TOL, err


@pytest.mark.parametrize("n,order,scheme", [(16, 5, "weno"), (14, 3, "tpp")])
def test_lake_rk_steps_match_oracle(n, order, scheme):
    print(f"case n={n} order={order} {scheme} lake over the cone (perturbed), 2 SSP-RK3 steps", flush=True)
    alpha, q, surface = _state("lake", n, 5)
    dt = cfl_dt(q)
    og, g = _grids(n, order, scheme, alpha, surface)
    ref = ssp_rk3(og.tendency, ssp_rk3(og.tendency, q, dt), dt)
    qp = to_padded(q, g.r)
    ws = g.workspace()
    for _ in range(2):
        g.rk_step(qp, dt, "ssp3", ws)
    torch.cuda.synchronize()
    err = rel_err(g.interior(qp), ref)
    print("rel err", err, flush=True)
    assert max(err) < TOL, err


def test_c_property_on_the_gpu_path():
    """The lake at rest over the kinked cone keeps the flat-bottom lake's
    residual tendency (C-property, section 2)."""
    from paper_2411_19185_amd import Grid
    n = 32
    cone = hi.ConeMountain()
    flat = lambda p: np.zeros(p.shape[:-1])
    res = []
    for surface in (cone, None):
        q = cell_average(hi.LakeAtRest(surface=surface or flat), n, A, nq=4)
        g = Grid(n, 5, "weno", surface=surface)
        dq = g.tendency(to_padded(q, g.r))
        torch.cuda.synchronize()
        res.append(float(dq.abs().max().cpu() / q[0].abs().max()))
    print("lake over the cone / flat bottom, max |dq/dt| / max q0:", res, flush=True)
    assert res[0] <= 1.05 * res[1]


def test_mountain_flow_five_days():
    """The section 5.2 case (zonal flow over the cone, h0 = 5960 m,
    u0 = 20 m/s) on C48 with WENO5 for five days: mass kept to round-off,
    thickness positive, everything finite."""
    from paper_2411_19185_amd import Grid
    n = 48
    a = hi.PAPER_RADIUS
    f = hi.MountainFlow(radius=a)
    q = cell_average(f, n, a, nq=4)
    g = Grid(n, 5, "weno", radius=a, surface=f.surface)
    dt = cfl_dt(q, radius=a)
    steps = int(math.ceil(5 * hi.DAY / dt))
    dt = 5 * hi.DAY / steps
    print(f"case C{n} WENO5 mountain flow, {steps} steps of {dt:.1f} s", flush=True)
    qp = to_padded(q, g.r)
    ws = g.workspace()
    m0 = float(q[0].sum())
    for _ in range(steps):
        g.rk_step(qp, dt, "ssp3", ws)
    torch.cuda.synchronize()
    assert g.bad_cells(qp) == 0
    m1 = float(g.interior(qp)[0].sum())
    print("relative mass change", abs(m1 - m0) / m0, flush=True)
    assert abs(m1 - m0) <= 2e-16 * steps * m0


def test_surface_that_is_not_finite_is_refused():
    from paper_2411_19185_amd import Grid
    from paper_2411_19185_amd._lib import HopeError
    with pytest.raises(HopeError) as e:
        Grid(8, 3, "tpp", surface=lambda p: np.full(p.shape[:-1], np.nan))
    assert "not finite" in str(e.value)


def _oracle_vjp(fn, q, w):
    qq = q.clone().requires_grad_(True)
    (fn(qq) * w).sum().backward()
    return qq.grad


VJP_CASES = [
    # (n, order, scheme, state, seed)
    (12, 3, "tpp", "mountain", 0),
    (10, 5, "weno", "mountain", 0),
    (9, 3, "weno", "ridge", 3),
    (12, 11, "tpp", "ridge", 4),
    (13, 5, "tpp", "lake", 5),
    (14, 7, "tpp", "mountain", 6),
]


@pytest.mark.parametrize("n,order,scheme,state,seed", VJP_CASES)
def test_tendency_vjp_with_topography_matches_oracle_autograd(n, order, scheme, state, seed):
    """The adjoint with topography: through sqrtG phi_t in the reconstruction,
    the pressure with phi_s and psi_B with its derivative reconstruction."""
    print(f"case n={n} order={order} {scheme} {state} (perturbed) seed={seed}: tendency adjoint", flush=True)
    alpha, q, surface = _state(state, n, seed)
    w = torch.tensor(hi.normal_array(seed + 500, tuple(q.shape)))
    og, g = _grids(n, order, scheme, alpha, surface)
    ref = _oracle_vjp(og.tendency, q, w)
    out = g.tendency_vjp(to_padded(q, g.r), w.cuda())
    torch.cuda.synchronize()
    err = rel_err(out, ref)
    print("rel err", err, flush=True)
    assert max(err) < TOL, err


@pytest.mark.parametrize("n,order,scheme,state,seed", [(12, 3, "tpp", "mountain", 7), (10, 5, "weno", "ridge", 8)])
def test_rk_step_vjp_with_topography_matches_oracle_autograd(n, order, scheme, state, seed):
    print(f"case n={n} order={order} {scheme} {state} (perturbed) seed={seed}: step adjoint", flush=True)
    alpha, q, surface = _state(state, n, seed)
    w = torch.tensor(hi.normal_array(seed + 500, tuple(q.shape)))
    dt = cfl_dt(q)
    og, g = _grids(n, order, scheme, alpha, surface)
    ref = _oracle_vjp(lambda x: ssp_rk3(og.tendency, x, dt), q, w)
    out = g.rk_step_vjp(to_padded(q, g.r), dt, w.cuda())
    torch.cuda.synchronize()
    err = rel_err(out, ref)
    print("rel err", err, flush=True)
    assert max(err) < TOL, err
