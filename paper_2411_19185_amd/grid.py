"""Torch-facing wrapper of the C ABI: a Grid owns a hope_grid handle and
passes tensor pointers and torch's current stream to the library."""
from __future__ import annotations

import ctypes
import os

import torch

from ._lib import (HOPE_ERR_NUMERIC, HOPE_OK, HOPE_PROFILE_SELECT, HOPE_RK_SSP3, HOPE_RK_WS3, Layout, check, lib,
                   make_desc, surface_callback)


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


class Grid:
    """One cubed-sphere grid (n cells per panel edge), reconstruction order
    and scheme ('tpp' or 'weno'), with the physical constants of the problem.
    surface: optional bottom topography, a callable p -> phi_s (surface
    geopotential at unit vectors p of shape (count, 3)), evaluated by the
    library while the grid is built."""

    def __init__(self, n: int, order: int, scheme: str = "tpp", radius: float = 6.371e6,
                 omega: float = 7.292e-5, axis_tilt: float = 0.0, weno_eps: float = 1e-12,
                 split_theta: float = 3.0, ghost_iters: int = 0, cache_dir: str | None = None, surface=None):
        if cache_dir is not None:
            cache_dir = os.path.expanduser(cache_dir)
            os.makedirs(cache_dir, exist_ok=True)
        cb = surface_callback(surface) if surface is not None else None
        self.desc = make_desc(n, order, scheme, radius, omega, axis_tilt, weno_eps, split_theta,
                              ghost_iters=ghost_iters, cache_dir=cache_dir, surface_fn=cb)
        h = ctypes.c_void_p()
        check(lib().hope_grid_create(ctypes.byref(self.desc), ctypes.byref(h)))
        self.surface = surface
        self._h = h
        lay = Layout()
        check(lib().hope_grid_layout(h, ctypes.byref(lay)))
        self.layout = lay
        self.n, self.order, self.scheme = n, order, scheme
        self.r = lay.r
        self.P = lay.padded
        self.m = lay.n_gauss

    def derive(self, axis_tilt: float) -> "Grid":
        """The same grid with another tilt of the rotation axis, sharing this
        grid's ghost map on the device (this grid is kept alive with it)."""
        h = ctypes.c_void_p()
        check(lib().hope_grid_derive(self._h, float(axis_tilt), ctypes.byref(h)))
        g = Grid.__new__(Grid)
        g.desc = make_desc(self.n, self.order, self.scheme, self.desc.radius, self.desc.omega, axis_tilt,
                           self.desc.weno_eps, self.desc.split_theta, ghost_iters=self.desc.ghost_iters)
        g._h = h
        g._base = self
        lay = Layout()
        check(lib().hope_grid_layout(h, ctypes.byref(lay)))
        g.layout = lay
        g.n, g.order, g.scheme = self.n, self.order, self.scheme
        g.r, g.P, g.m = self.r, self.P, self.m
        return g

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().hope_grid_destroy(h)
            self._h = None

    # ------------------------------------------------------------------
    def new_state(self, device="cuda") -> torch.Tensor:
        return torch.zeros(3, 6, self.P, self.P, dtype=torch.float64, device=device)

    def interior(self, q: torch.Tensor) -> torch.Tensor:
        r, n = self.r, self.n
        return q[:, :, r:r + n, r:r + n]

    def _check_padded(self, q):
        if not (q.is_cuda and q.dtype == torch.float64 and q.is_contiguous()
                and tuple(q.shape) == (3, 6, self.P, self.P)):
            raise ValueError(f"state must be a contiguous cuda float64 tensor of shape (3, 6, {self.P}, {self.P})")

    def _check_field(self, f):
        if not (f.is_cuda and f.dtype == torch.float64 and f.is_contiguous()
                and tuple(f.shape) == (3, 6, self.n, self.n)):
            raise ValueError(f"field must be a contiguous cuda float64 tensor of shape (3, 6, {self.n}, {self.n})")

    # ------------------------------------------------------------------
    def bad_cells(self, q: torch.Tensor) -> int:
        """Number of interior cells of the padded state q whose thickness is
        not positive or whose variables are not finite (waits for the
        current stream)."""
        self._check_padded(q)
        n_bad = ctypes.c_int64()
        code = lib().hope_check_state(self._h, _ptr(q), ctypes.byref(n_bad), _stream())
        if code not in (HOPE_OK, HOPE_ERR_NUMERIC):
            check(code)
        return n_bad.value

    def fill_halo(self, q: torch.Tensor) -> torch.Tensor:
        self._check_padded(q)
        check(lib().hope_fill_halo(self._h, _ptr(q), _stream()))
        return q

    def tendency(self, q: torch.Tensor, out: torch.Tensor | None = None,
                 ws: torch.Tensor | None = None) -> torch.Tensor:
        """dq/dt (interior) of the padded state q; its ghost rings are
        overwritten.  ws: scratch of tendency_workspace() size, else one is
        allocated for the call."""
        self._check_padded(q)
        if out is None:
            out = torch.empty(3, 6, self.n, self.n, dtype=torch.float64, device=q.device)
        self._check_field(out)
        if ws is None:
            ws = self.tendency_workspace()
        check(lib().hope_tendency(self._h, _ptr(q), _ptr(out), _ptr(ws), ws.numel() * 8, _stream()))
        return out

    def tendency_vjp(self, q: torch.Tensor, w: torch.Tensor, out: torch.Tensor | None = None,
                     ws: torch.Tensor | None = None) -> torch.Tensor:
        """dL/dq (interior) of the tendency at the padded state q, given
        w = dL/d(dq/dt)."""
        self._check_padded(q)
        self._check_field(w)
        if out is None:
            out = torch.empty(3, 6, self.n, self.n, dtype=torch.float64, device=q.device)
        self._check_field(out)
        if ws is None:
            ws = self.vjp_workspace()
        check(lib().hope_tendency_vjp(self._h, _ptr(q), _ptr(w), _ptr(out), _ptr(ws), ws.numel() * 8, _stream()))
        return out

    def tendency_workspace(self) -> torch.Tensor:
        return torch.empty(self.layout.tendency_workspace_bytes // 8, dtype=torch.float64, device="cuda")

    def workspace(self) -> torch.Tensor:
        return torch.empty(self.layout.rk_workspace_bytes // 8, dtype=torch.float64, device="cuda")

    def vjp_workspace(self) -> torch.Tensor:
        return torch.empty(self.layout.vjp_workspace_bytes // 8, dtype=torch.float64, device="cuda")

    def rk_vjp_workspace(self) -> torch.Tensor:
        return torch.empty(self.layout.rk_vjp_workspace_bytes // 8, dtype=torch.float64, device="cuda")

    def rk_step(self, q: torch.Tensor, dt: float, scheme: str = "ssp3", ws: torch.Tensor | None = None):
        self._check_padded(q)
        if ws is None:
            ws = self.workspace()
        code = {"ssp3": HOPE_RK_SSP3, "ws3": HOPE_RK_WS3}[scheme]
        check(lib().hope_rk_step(self._h, _ptr(q), float(dt), code, _ptr(ws), ws.numel() * 8, _stream()))
        return q

    def rk_step_vjp(self, q: torch.Tensor, dt: float, gout: torch.Tensor, scheme: str = "ssp3",
                    out: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
        """dL/dq^n of one RK step from q^n (padded) and gout = dL/dq^{n+1}."""
        self._check_padded(q)
        self._check_field(gout)
        if out is None:
            out = torch.empty(3, 6, self.n, self.n, dtype=torch.float64, device=q.device)
        self._check_field(out)
        if ws is None:
            ws = self.rk_vjp_workspace()
        code = {"ssp3": HOPE_RK_SSP3, "ws3": HOPE_RK_WS3}[scheme]
        check(lib().hope_rk_step_vjp(self._h, _ptr(q), float(dt), code, _ptr(gout), _ptr(out), _ptr(ws),
                                     ws.numel() * 8, _stream()))
        return out

    def set_launch(self, strip_w: int, seg_h: int):
        """The stage kernel's launch shape; the workspace sizes depend on
        seg_h (segment seams), so the layout is read again."""
        check(lib().hope_grid_set_launch(self._h, int(strip_w), int(seg_h)))
        lay = Layout()
        check(lib().hope_grid_layout(self._h, ctypes.byref(lay)))
        self.layout = lay

    def get_launch(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        check(lib().hope_grid_get_launch(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    # ------------------------------------------------------------------
    KERNELS = {"fill_halo": 0, "edge_traces": 1, "stage": 2, "vjp_traces": 3, "vjp_points": 4, "vjp_edges": 5,
               "vjp_weno": 6, "vjp_gather": 7, "vjp_ghost_t": 8}

    def profile(self, enable: bool, only: tuple[str, ...] | None = None):
        """Start (clearing the record) or stop per-kernel timing; with ``only``,
        just those kernels are bracketed by events."""
        if not enable:
            code = 0
        elif only is None:
            code = 1
        else:
            code = HOPE_PROFILE_SELECT
            for name in only:
                code |= 1 << self.KERNELS[name]
        check(lib().hope_grid_profile(self._h, code))

    def profile_read(self, kernel: str):
        """(total ms, launches) of one kernel since profile(True)."""
        ms, cnt = ctypes.c_double(), ctypes.c_int64()
        check(lib().hope_grid_profile_read(self._h, self.KERNELS[kernel], ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value
