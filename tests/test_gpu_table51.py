"""The paper's accuracy experiment (section 5.1, Table 5.1) on the GPU path:
the steady-state geostrophic flow integrated for 12 days with the paper's
three-stage Runge-Kutta scheme and time steps, with TPP3 to TPP11 at C30 to
C360.  The paper ran in quadruple precision; FP64 rounding, accumulated over
up to 2e4 steps of relative error 1.1e-16 each, adds up to about 1e-14 to a
normalised error, so the cases kept are those whose printed errors lie above
that floor (all of TPP3 and TPP5, TPP7 to C90, TPP9 and TPP11 to C45).

Each normalised geopotential error must equal the printed one to within half
a unit of its fifth printed digit plus that floor, 1e-14 absolute.  Where the
printed error exceeds about 2e-10 the floor is below the fifth digit, and
this is agreement to the five printed digits.  Below that (TPP7 at C90, TPP9
and TPP11 at C45) the floor dominates and the check is weaker: TPP11 C45
L-infinity agrees to four digits only (2.8594e-12 against 2.8579e-12).
There the convergence rates, checked to 2e-3 against the printed ones at
every resolution pair, are what hold the result.
This pins the readings the path shares with the oracle end to end, including
the second stage of (3.40) taken from q^n, and the high-order kernels."""
import math

import numpy as np
import pytest
import torch

import hope_inputs as hi
from golden.table51 import DT, load
from oracle.ic import cell_average, cell_sqrt_g
from oracle.norms import error_norms

pytestmark = pytest.mark.gpu

DAY = 86400.0


def _run(order, n):
    from paper_2411_19185_amd import Grid
    a = hi.PAPER_RADIUS
    q0 = cell_average(hi.BalancedFlow(alpha=0.0, radius=a), n, a, nq=4)
    g = Grid(n, order, "tpp", radius=a, axis_tilt=0.0)
    qp = g.new_state()
    g.interior(qp).copy_(q0.cuda())
    ws = g.workspace()
    steps = int(round(12 * DAY / DT[n]))
    for _ in range(steps):
        g.rk_step(qp, DT[n], "ws3", ws)
    torch.cuda.synchronize()
    sg = cell_sqrt_g(n, a)[None, :, :]
    phi = g.interior(qp)[0].cpu().numpy() / sg
    ref = q0[0].numpy() / sg
    l1, l2, linf = error_norms(phi, ref, np.broadcast_to(sg, phi.shape))
    return {"L1": l1, "L2": l2, "Linf": linf}


# resolutions per order whose printed errors lie above the FP64 floor
CASES = {3: (30, 45, 90, 180, 360), 5: (30, 45, 90, 180, 360), 7: (30, 45, 90), 9: (30, 45), 11: (30, 45)}
FP64_FLOOR = 1e-14


@pytest.mark.parametrize("order", sorted(CASES))
def test_table_5_1_rates_and_errors(order):
    errors, rates = load()
    key = f"tpp{order}"
    res = CASES[order]
    got = {}
    for n in res:
        print(f"case TPP{order} C{n}, 12 days", flush=True)
        got[n] = _run(order, n)
        print("  ", got[n], "paper", {nm: errors[(key, nm)][n] for nm in ("L1", "L2", "Linf")}, flush=True)
    for norm in ("L1", "L2", "Linf"):
        for n in res:
            printed = errors[(key, norm)][n]
            # half a unit of the fifth printed digit (<= 5e-5 relative) plus the FP64 floor
            assert abs(got[n][norm] - printed) <= 5.1e-5 * printed + FP64_FLOOR, (norm, n, got[n][norm], printed)
        for a, b in zip(res, res[1:]):
            printed = rates[(key, norm)][b]
            rate = math.log(got[a][norm] / got[b][norm]) / math.log(b / a)
            print(f"  rate {norm} C{a}->C{b}: {rate:.4f} (paper {printed})", flush=True)
            assert abs(rate - printed) < 2e-3, (norm, a, b, rate, printed)
