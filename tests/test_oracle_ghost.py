"""Pins of the oracle's ghost-cell fill (section 3.3.1, appendix (7.1)-(7.12))."""
import numpy as np
import pytest
import torch

import hope_inputs as hi
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
