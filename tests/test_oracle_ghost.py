"""Pins of the oracle's ghost-cell fill (section 3.3.1, appendix (7.1)-(7.12))."""
import math

import numpy as np
import pytest
import torch

import hope_inputs as hi
from oracle import geometry as geo
from oracle.ghost import GhostMap
from oracle.ic import cell_average

A = 6.371e6


@pytest.mark.parametrize("n,k", [(4, 3), (6, 5)])
def test_fixed_point_equals_direct_solve(n, k):
    """The converged iteration equals the solution of (I - C) v = A-bar q
    assembled densely and solved directly ((7.10)-(7.12))."""
    gm = GhostMap(n, k, A)
    q = torch.rand(3, 6, n, n, dtype=torch.float64, generator=torch.Generator().manual_seed(0)) + 0.5
    a = gm.fill(q)
    b = gm.dense_solve(q)
    assert float((a - b).abs().max() / b.abs().max()) < 1e-14
    assert gm.sweeps_used < 40


def test_linearity():
    """(7.12): the ghost values are a linear map of the interior values."""
    n, k = 8, 5
    gm = GhostMap(n, k, A)
    g = torch.Generator().manual_seed(1)
    q1 = torch.rand(3, 6, n, n, dtype=torch.float64, generator=g)
    q2 = torch.rand(3, 6, n, n, dtype=torch.float64, generator=g)
    lhs = gm.fill(2.5 * q1 - 1.5 * q2)
    rhs = 2.5 * gm.fill(q1) - 1.5 * gm.fill(q2)
    assert float((lhs - rhs).abs().max() / rhs.abs().max()) < 1e-14


def test_paper_fixed_count_close_to_fixed_point():
    """Ten sweeps (the paper's fixed count) are already close to the fixed point."""
    n, k = 10, 5
    gm = GhostMap(n, k, A)
    q = cell_average(hi.BalancedFlow(alpha=0.4), n, A, nq=4)
    a = gm.fill(q)
    b = gm.fill(q, sweeps=10)
    for v in range(3):
        assert float((a[v] - b[v]).abs().max() / a[v].abs().max()) < 1e-7


@pytest.mark.parametrize("k", [3, 5])
def test_ghost_values_converge_at_design_order(k):
    """Ghost values of a smooth state approach the exact averages over the
    extended cells at order k, for mass and both momentum components (a
    wrong owner, stencil or conversion would leave an O(1) error)."""
    f = hi.BalancedFlow(alpha=0.6)
    errs = []
    for n in (20, 40):
        gm = GhostMap(n, k, A)
        r = gm.r
        q = cell_average(f, n, A, nq=8)
        exact = cell_average(f, n, A, nq=8, pad=r)
        got = gm.fill(q)
        mask = torch.ones(gm.P, gm.P, dtype=torch.bool)
        mask[r:r + n, r:r + n] = False
        e = [(got[v][:, mask] - exact[v][:, mask]).abs().max() / exact[v].abs().max() for v in range(3)]
        errs.append(np.array([float(x) for x in e]))
    rate = np.log2(errs[0] / errs[1])
    assert (rate > k - 0.35).all(), rate
    assert (errs[1] < 1e-3).all()


def test_fixed_point_converges_for_order_11_on_12_cells():
    gm = GhostMap(12, 11, A)
    q = cell_average(hi.BalancedFlow(alpha=0.2), 12, A, nq=4)
    gm.fill(q)
    assert gm.sweeps_used < 40


def _rotation_image(n, r, R):
    """Where the cube rotation R sends each padded cell, and its frame.

    For panel p the image panel p' is the one whose axis is R times p's axis;
    the cell (jj, ii) goes to the padded cell of p' holding R times its
    centre, and the contravariant wind (u, v) to M_p (u, v), from R applied to
    the two coordinate tangent vectors (a signed permutation here)."""
    P = n + 2 * r
    d = 0.5 * math.pi / n
    cen = geo.cell_centres(n, r) * d
    xx, yy = np.meshgrid(cen, cen, indexing="xy")                 # [jj, ii]
    dest, frames = [], []
    for p in range(6):
        pp = int(np.argmax(geo.PANEL_AXIS @ (R @ geo.PANEL_AXIS[p])))
        w = geo.panel_xyz(p, np.tan(xx), np.tan(yy)) @ R.T
        Xp, Yp = geo.xyz_to_XY(pp, w)
        ii = np.rint(np.arctan(Xp) / d + n / 2.0 - 0.5 + r).astype(int)
        jj = np.rint(np.arctan(Yp) / d + n / 2.0 - 0.5 + r).astype(int)
        assert np.abs(np.arctan(Xp) / d + n / 2.0 - 0.5 + r - ii).max() < 1e-9
        dest.append((pp, jj, ii))
        # tangents at the panel centre by central differences
        h = 1e-6
        tang = lambda q_, x, y: np.stack([(geo.panel_xyz(q_, np.tan(x + h), np.tan(y)) -
                                           geo.panel_xyz(q_, np.tan(x - h), np.tan(y))) / (2 * h),
                                          (geo.panel_xyz(q_, np.tan(x), np.tan(y + h)) -
                                           geo.panel_xyz(q_, np.tan(x), np.tan(y - h))) / (2 * h)], -1)
        E = tang(p, 0.0, 0.0)                    # columns e_x, e_y of p (3 x 2)
        c = R @ geo.panel_xyz(p, 0.0, 0.0)
        Xc, Yc = geo.xyz_to_XY(pp, c)
        Ep = tang(pp, float(np.arctan(Xc)), float(np.arctan(Yc)))
        M = np.linalg.lstsq(Ep, R @ E, rcond=None)[0]          # R E = Ep M
        Mi = np.rint(M)
        assert np.abs(M - Mi).max() < 1e-6
        frames.append(Mi)
    return dest, frames


def _rotate_padded(qp, dest, frames):
    out = torch.zeros_like(qp)
    for p in range(6):
        pp, jj, ii = dest[p]
        M = frames[p]
        src = qp[:, p]
        out[0, pp, jj, ii] = src[0]
        out[1, pp, jj, ii] = M[0, 0] * src[1] + M[0, 1] * src[2]
        out[2, pp, jj, ii] = M[1, 0] * src[1] + M[1, 1] * src[2]
    return out


@pytest.mark.parametrize("n,k", [(6, 3), (7, 5)])
@pytest.mark.parametrize("axis", ["z", "x"])
def test_ghost_fill_commutes_with_cube_rotations(n, k, axis):
    """Rotating the interior state by a symmetry of the cube and then filling
    the ghosts gives the rotation of the filled state, ghost rings and corner
    blocks included, mass and both momentum components (the 90-degree turns
    about z and x generate all 24 rotations).  A wrong owner panel, stencil
    or conversion on any panel edge breaks this."""
    R = {"z": np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]]),
         "x": np.array([[1.0, 0.0, 0.0], [0.0, 0.0, -1.0], [0.0, 1.0, 0.0]])}[axis]
    gm = GhostMap(n, k, A)
    r = gm.r
    dest, frames = _rotation_image(n, r, R)
    g = torch.Generator().manual_seed(7)
    q = torch.rand(3, 6, n, n, dtype=torch.float64, generator=g) + 0.5
    qpad = torch.zeros(3, 6, n + 2 * r, n + 2 * r, dtype=torch.float64)
    qpad[:, :, r:r + n, r:r + n] = q
    q_rot = _rotate_padded(qpad, dest, frames)[:, :, r:r + n, r:r + n]
    lhs = gm.fill(q_rot)
    rhs = _rotate_padded(gm.fill(q), dest, frames)
    for v in range(3):
        assert float((lhs[v] - rhs[v]).abs().max() / rhs[v].abs().max()) < 1e-13
