"""Batched ensembles: members of one order and scheme on grids of uneven
resolutions, advanced together by the library's batched kernels (one launch
per kernel over all members), optionally as one captured HIP graph per
Runge-Kutta step.

    grids = {n: Grid(n, 5, "weno") for n in (48, 64, 90, 128)}
    ens = Ensemble([grids[n] for n in sizes], axis_tilt=tilts)
    q = ens.new_state();  ens.member_interior(q, i).copy_(...)
    dt = torch.tensor(per_member_dt, device="cuda", dtype=torch.float64)
    step = ens.capture_step(q, dt)      # a torch.cuda.CUDAGraph
    for _ in range(steps): step.replay()
"""
from __future__ import annotations

import ctypes

import torch

from ._lib import HOPE_RK_SSP3, HOPE_RK_WS3, BatchInfo, check, lib
from .grid import Grid, _ptr, _stream

_SCHEMES = {"ssp3": HOPE_RK_SSP3, "ws3": HOPE_RK_WS3}


class Ensemble:
    """members[i] runs on grids[i] (grids may repeat); axis_tilt gives each
    member its own rotation-axis tilt (radians), else each grid's own."""

    def __init__(self, grids: list[Grid], axis_tilt: list[float] | None = None):
        n = len(grids)
        if n == 0:
            raise ValueError("an ensemble needs at least one member")
        self.grids = list(grids)       # the grids must outlive the batch
        self.axis_tilt = list(axis_tilt) if axis_tilt is not None else None
        self._member_grids: dict[int, Grid] = {}
        self._private_grids: dict[int, Grid] = {}
        self._streams: list = []
        arr = (ctypes.c_void_p * n)(*[g._h.value for g in grids])
        tilt = (ctypes.c_double * n)(*axis_tilt) if axis_tilt is not None else None
        h = ctypes.c_void_p()
        check(lib().hope_batch_create(arr, n, tilt, ctypes.byref(h)))
        self._h = h
        self.n_members = n
        self._refresh()

    def _refresh(self):
        info = BatchInfo()
        so = (ctypes.c_int64 * self.n_members)()
        fo = (ctypes.c_int64 * self.n_members)()
        check(lib().hope_batch_layout(self._h, ctypes.byref(info), so, fo))
        self.info = info
        self.state_offsets = list(so)
        self.field_offsets = list(fo)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().hope_batch_destroy(h)
            self._h = None

    # ------------------------------------------------------------------
    def new_state(self) -> torch.Tensor:
        return torch.zeros(self.info.state_elems, dtype=torch.float64, device="cuda")

    def new_field(self) -> torch.Tensor:
        return torch.empty(self.info.field_elems, dtype=torch.float64, device="cuda")

    def workspace(self) -> torch.Tensor:
        return torch.empty(self.info.rk_workspace_bytes // 8, dtype=torch.float64, device="cuda")

    def member_state(self, q_all: torch.Tensor, i: int) -> torch.Tensor:
        g = self.grids[i]
        o = self.state_offsets[i]
        return q_all[o:o + 18 * g.P * g.P].view(3, 6, g.P, g.P)

    def member_interior(self, q_all: torch.Tensor, i: int) -> torch.Tensor:
        return self.grids[i].interior(self.member_state(q_all, i))

    def member_field(self, f_all: torch.Tensor, i: int) -> torch.Tensor:
        g = self.grids[i]
        o = self.field_offsets[i]
        return f_all[o:o + 18 * g.n * g.n].view(3, 6, g.n, g.n)

    def _check(self, t: torch.Tensor, elems: int, what: str):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() >= elems):
            raise ValueError(f"{what} must be a contiguous cuda float64 tensor of at least {elems} elements")

    # ------------------------------------------------------------------
    def tendency(self, q_all: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._check(q_all, self.info.state_elems, "q_all")
        if out is None:
            out = self.new_field()
        self._check(out, self.info.field_elems, "out")
        check(lib().hope_batch_tendency(self._h, _ptr(q_all), _ptr(out), _stream()))
        return out

    def rk_stage(self, stage: int, q_all: torch.Tensor, dt: torch.Tensor, ws: torch.Tensor, scheme: str = "ssp3"):
        self._check(q_all, self.info.state_elems, "q_all")
        self._check(dt, self.n_members, "dt")
        check(lib().hope_batch_rk_stage(self._h, int(stage), _SCHEMES[scheme], _ptr(q_all), _ptr(dt), _ptr(ws),
                                        ws.numel() * 8, _stream()))

    def rk_step(self, q_all: torch.Tensor, dt: torch.Tensor, ws: torch.Tensor | None = None,
                scheme: str = "ssp3") -> torch.Tensor:
        """One Runge-Kutta step of every member, in place; dt: per-member time
        steps (cuda float64, read when the step runs)."""
        self._check(q_all, self.info.state_elems, "q_all")
        self._check(dt, self.n_members, "dt")
        if ws is None:
            ws = self.workspace()
        check(lib().hope_batch_rk_step(self._h, _SCHEMES[scheme], _ptr(q_all), _ptr(dt), _ptr(ws), ws.numel() * 8,
                                       _stream()))
        return q_all

    def capture_step(self, q_all: torch.Tensor, dt: torch.Tensor, ws: torch.Tensor | None = None,
                     scheme: str = "ssp3") -> torch.cuda.CUDAGraph:
        """A HIP graph of one Runge-Kutta step on these buffers (12 kernel
        launches at WENO5 and TPP9+, 9 at the other orders; no memory
        operations).  Replaying it advances q_all in
        place with the values dt holds at replay time."""
        if ws is None:
            ws = self.workspace()
        # one eager evaluation first, so that every kernel is loaded before
        # capture (it writes only the ghost rings of q_all and a scratch field)
        self.tendency(q_all)
        torch.cuda.synchronize()
        self._graph_buffers = (q_all, dt, ws)      # kept alive with the graph
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            self.rk_step(q_all, dt, ws, scheme)
        # the graph refers to this batch's device tables: it keeps the ensemble
        # (and with it the batch and its grids) alive; the batch's launch shape
        # is fixed from now on (hope_batch_set_launch refuses)
        graph._hope_ensemble = self
        return graph

    def member_grid(self, i: int) -> Grid:
        """A single-grid handle for member i (its grid with its own axis tilt,
        sharing the grid's ghost map), for per-member work such as adjoints."""
        if i not in self._member_grids:
            g = self.grids[i]
            self._member_grids[i] = g if self.axis_tilt is None else g.derive(self.axis_tilt[i])
        return self._member_grids[i]

    def member_loss_gradient(self, i: int, q0: torch.Tensor, dt: float, steps: int, checkpoint_every: int = 5,
                             scheme: str = "ssp3") -> torch.Tensor:
        """d/dq0 of 0.5 ||q_T||^2 for member i after ``steps`` Runge-Kutta steps
        from its interior state q0 (3, 6, n, n): checkpointed forward, then the
        hand-written step adjoints in reverse."""
        from .autograd import rollout
        q = q0.detach().clone().requires_grad_(True)
        qT = rollout(self.member_grid(i), q, dt, steps, checkpoint_every, scheme)
        (0.5 * (qT * qT).sum()).backward()
        return q.grad

    def member_loss_gradients(self, q0s: list[torch.Tensor], dts: list[float], steps: int,
                              checkpoint_every: int = 5, scheme: str = "ssp3",
                              streams: int = 4) -> list[torch.Tensor]:
        """member_loss_gradient for every member, with the members spread over
        ``streams`` HIP streams (default priority) so that the launches of
        small members overlap on the GPU.  Each member runs on a grid handle of
        its own (its panel-edge trace scratch is private), and each stream on
        its own workspaces; results equal the one-by-one ones bitwise."""
        from .autograd import rollout
        n = self.n_members
        if len(q0s) != n or len(dts) != n:
            raise ValueError("one initial state and one time step per member")
        handles = []
        for i in range(n):
            if self.axis_tilt is not None:
                handles.append(self.member_grid(i))
            else:
                if i not in self._private_grids:
                    self._private_grids[i] = self.grids[i].derive(self.grids[i].desc.axis_tilt)
                handles.append(self._private_grids[i])
        main = torch.cuda.current_stream()
        # the pool persists across calls, so that the caching allocator's
        # per-stream blocks are reused
        while len(self._streams) < max(1, int(streams)):
            self._streams.append(torch.cuda.Stream())
        pool = self._streams[:max(1, int(streams))]
        for st in pool:
            st.wait_stream(main)
        grads = []
        for i in range(n):
            st = pool[i % len(pool)]
            with torch.cuda.stream(st):
                q = q0s[i].detach().clone().requires_grad_(True)
                qT = rollout(handles[i], q, dts[i], steps, checkpoint_every, scheme)
                (0.5 * (qT * qT).sum()).backward()
                grads.append(q.grad)
        for st in pool:
            main.wait_stream(st)
        for gr in grads:
            gr.record_stream(main)
        return grads

    # ------------------------------------------------------------------
    def set_launch(self, strip_w: list[int] | None = None, seg_h: list[int] | None = None, blocks: int = 0):
        sw = (ctypes.c_int32 * self.n_members)(*strip_w) if strip_w is not None else None
        sh = (ctypes.c_int32 * self.n_members)(*seg_h) if seg_h is not None else None
        check(lib().hope_batch_set_launch(self._h, sw, sh, int(blocks)))
        self._refresh()

    def get_launch(self):
        sw = (ctypes.c_int32 * self.n_members)()
        sh = (ctypes.c_int32 * self.n_members)()
        b = ctypes.c_int32()
        check(lib().hope_batch_get_launch(self._h, sw, sh, ctypes.byref(b)))
        return list(sw), list(sh), b.value
