"""GPU test of the per-kernel timing: every kernel, or only selected ones,
is bracketed by events (the fused stage's recorded by its own launches, with
and without the seam kernel), and timing does not change results."""
import ctypes

import pytest
import torch

from cases import STATES, cfl_dt, to_padded

pytestmark = pytest.mark.gpu


def test_profile_all_or_selected_kernels():
    from paper_2411_19185_amd import Grid
    from paper_2411_19185_amd._lib import HOPE_PROFILE_SELECT, lib
    n = 24
    alpha, q = STATES["member"](n, 3, nq=2)
    g = Grid(n, 5, "weno", axis_tilt=alpha)
    qp = to_padded(q, g.r)
    ref = g.tendency(qp)
    g.profile(True)
    a = g.tendency(qp)
    g.profile(False)
    assert [g.profile_read(k)[1] for k in ("fill_halo", "edge_traces", "stage")] == [1, 1, 1]
    assert all(g.profile_read(k)[0] > 0 for k in ("fill_halo", "edge_traces", "stage"))
    g.profile(True, only=("stage",))
    b = g.tendency(qp)
    b2 = g.tendency(qp)
    g.profile(False)
    assert [g.profile_read(k)[1] for k in ("fill_halo", "edge_traces", "stage")] == [0, 0, 2]
    # one segment per panel: no seam kernel, the stage kernel records both events
    g.set_launch(30, n)
    g.profile(True, only=("stage",))
    c = g.tendency(qp)
    g.profile(False)
    ms, cnt = g.profile_read("stage")
    assert cnt == 1 and ms > 0
    torch.cuda.synchronize()
    assert torch.equal(a, ref) and torch.equal(b, ref) and torch.equal(b2, ref) and torch.equal(c, ref)
    # codes other than 0, 1 and HOPE_PROFILE_SELECT | kernel bits are rejected
    assert lib().hope_grid_profile(g._h, 2) == -1
    assert lib().hope_grid_profile(g._h, HOPE_PROFILE_SELECT | (1 << 12)) == -1
    assert lib().hope_grid_profile(g._h, 0) == 0


def test_captured_rk_steps_with_stage_timing_on_equal_eager_steps():
    """hope_rk_step recorded in a HIP graph while the stage is being timed
    (timing steps aside under stream capture): every replay, with eager steps
    and synchronisations between the replays, equals the eager steps bitwise."""
    from paper_2411_19185_amd import Grid
    n = 24
    alpha, q = STATES["member"](n, 5, nq=2)
    g = Grid(n, 5, "weno", axis_tilt=alpha)
    dt = cfl_dt(q)
    ws, ws_eager = g.workspace(), g.workspace()
    q_graph = to_padded(q, g.r)
    q_eager = q_graph.clone()
    g.profile(True, only=("stage",))
    g.rk_step(q_graph.clone(), dt, "ssp3", ws)      # loads the kernels before capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g.rk_step(q_graph, dt, "ssp3", ws)
    g.profile(False)
    for k in range(3):
        graph.replay()
        g.rk_step(q_eager, dt, "ssp3", ws_eager)
        torch.cuda.synchronize()
        assert torch.equal(q_graph, q_eager), k
