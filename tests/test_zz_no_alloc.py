"""hope_rk_step_static, the Runge-Kutta step whose workspace is a static
device array (for callers that cannot allocate), against hope_rk_step with a
caller workspace, through the C ABI: bitwise equal results on consecutive
calls, the later ones on a smaller grid (the array keeps the earlier call's
contents), and a clear refusal for a grid whose workspace does not fit."""
import ctypes

import pytest
import torch

from cases import STATES, cfl_dt, to_padded

pytestmark = pytest.mark.gpu


def _static_step(g, q, dt, scheme):
    from paper_2411_19185_amd._lib import HOPE_RK_SSP3, HOPE_RK_WS3, lib
    code = {"ssp3": HOPE_RK_SSP3, "ws3": HOPE_RK_WS3}[scheme]
    return lib().hope_rk_step_static(g._h, ctypes.c_void_p(q.data_ptr()), float(dt), code,
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def test_static_rk_step_matches_workspace_step():
    from paper_2411_19185_amd import Grid
    for n, order, scheme, seed, rk in [(96, 5, "weno", 90, "ssp3"), (40, 11, "tpp", 91, "ssp3"),
                                       (24, 5, "tpp", 92, "ws3")]:
        print(f"case n={n} order={order} {scheme} {rk}: static-scratch step vs workspace step", flush=True)
        alpha, q = STATES["member"](n, seed)
        g = Grid(n, order, scheme, axis_tilt=alpha)
        dt = cfl_dt(q)
        a = to_padded(q, g.r)
        b = a.clone()
        ws = g.workspace()
        for _ in range(2):
            g.rk_step(a, dt, rk, ws)
            assert _static_step(g, b, dt, rk) == 0
        torch.cuda.synchronize()
        assert torch.equal(g.interior(a), g.interior(b))


def test_static_rk_step_refuses_a_grid_too_large():
    from paper_2411_19185_amd import Grid
    from paper_2411_19185_amd._lib import lib
    n = 400
    print(f"case n={n} WENO5, two-row segments: workspace beyond the static scratch", flush=True)
    g = Grid(n, 5, "weno")
    g.set_launch(30, 2)                       # the segment seams' scratch grows as segments shrink
    assert g.layout.rk_workspace_bytes > 128 << 20
    q = g.new_state()
    assert _static_step(g, q, 1.0, "ssp3") == -1
    assert b"static scratch" in lib().hope_last_error()
