"""MI355X (gfx950) implementation of the HOPE cubed-sphere shallow-water
right-hand side (arXiv 2411.19185): hand-written HIP kernels behind the C ABI
of include/hope.h, with a thin torch binding.

    from paper_2411_19185_amd import Grid
    g = Grid(360, 5, "weno")
    q = g.new_state();  ...fill g.interior(q)...
    dqdt = g.tendency(q)
"""
from ._lib import HopeError, header_functions, inspect_ghost_map, lib  # noqa: F401
from .grid import Grid  # noqa: F401

__all__ = ["Grid", "HopeError", "lib", "header_functions", "inspect_ghost_map"]
