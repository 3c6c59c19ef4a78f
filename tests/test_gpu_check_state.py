"""GPU tests of the state check: the count of interior cells whose thickness
is not positive or whose variables are not finite equals the same count taken
on the host, ghost rings are ignored, and a checked rollout names the step at
which the state went bad."""
import ctypes

import pytest
import torch

from cases import STATES, to_padded

pytestmark = pytest.mark.gpu


def _host_count(q):
    h, mu, mv = q[0], q[1], q[2]
    bad = ~(h > 0) | ~torch.isfinite(h) | ~torch.isfinite(mu) | ~torch.isfinite(mv)
    return int(bad.sum())


@pytest.mark.parametrize("n,order,seed", [(13, 5, 0), (90, 3, 1), (360, 5, 2)])
def test_bad_cell_count_equals_host_count(n, order, seed):
    from paper_2411_19185_amd import Grid
    from paper_2411_19185_amd._lib import lib
    print(f"case n={n} order={order} seed={seed}", flush=True)
    g = Grid(n, order, "tpp")
    _, q = STATES["member"](n, seed)
    qp = to_padded(q, g.r)
    assert g.bad_cells(qp) == 0
    # plant bad values: zero and negative thickness, NaN and infinite momentum
    gen = torch.Generator().manual_seed(seed)
    cells = torch.randperm(6 * n * n, generator=gen)[:40]
    planted = [0.0, -1.0, float("nan"), float("inf"), -float("inf")]
    for t, c in enumerate(cells.tolist()):
        f, rem = divmod(c, n * n)
        j, i = divmod(rem, n)
        var = 0 if t % 3 == 0 else 1 + t % 2
        val = planted[t % len(planted)]
        if var > 0 and val in (0.0, -1.0):
            val = float("nan")
        q[var, f, j, i] = val
    qp = to_padded(q, g.r)
    # ghost rings are not part of the state
    r = g.r
    qp[:, :, :r, :] = float("nan")
    qp[0, :, -r:, :] = -1.0
    expect = _host_count(q)
    assert 0 < expect <= 40
    assert g.bad_cells(qp) == expect
    nb = ctypes.c_int64()
    rc = lib().hope_check_state(g._h, ctypes.c_void_p(qp.data_ptr()), ctypes.byref(nb), None)
    assert rc == -5 and nb.value == expect
    assert str(expect) in lib().hope_last_error().decode()


def test_check_state_rejects_null():
    from paper_2411_19185_amd import Grid
    from paper_2411_19185_amd._lib import lib
    g = Grid(12, 3, "tpp")
    nb = ctypes.c_int64(7)
    assert lib().hope_check_state(g._h, None, ctypes.byref(nb), None) == -1
    assert nb.value == 0
    assert lib().hope_check_state(None, None, None, None) == -1


def test_checked_rollout_names_the_step():
    from paper_2411_19185_amd import Grid
    from paper_2411_19185_amd import autograd as ad
    from cases import cfl_dt
    n = 16
    g = Grid(n, 3, "tpp")
    _, q = STATES["member"](n, 3)
    qg = q.cuda()
    dt = cfl_dt(q)
    out = ad.rollout(g, qg, dt, 4, checkpoint_every=2, check_state=True)
    assert g.bad_cells(to_padded(out.cpu(), g.r)) == 0
    qg[1, 2, 5, 5] = float("nan")
    with pytest.raises(FloatingPointError, match="after step 2"):
        ad.rollout(g, qg, dt, 4, checkpoint_every=2, check_state=True)
