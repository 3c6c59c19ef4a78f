"""Ghost-cell interpolation across panel edges (section 3.3, appendix (7.1)-(7.12)).
Test infrastructure only.

The padded array of a panel holds r = (k-1)/2 layers of ghost cells around
its n x n interior, corner blocks included (Figure 3.1b).  A ghost cell of
panel A is filled as follows (section 3.3.1):

 1. each of its m x m Gauss quadrature points (GQPs) is a point of A's
    extended gnomonic coordinates; its direction on the sphere lies in an
    owner panel B (largest signed Cartesian component; on an exact tie the
    two owners are averaged);
 2. the point value there is the order-k TPP reconstruction in B, on the
    central k x k stencil around the B cell that contains the point, read
    from B's *padded* array (so B's own ghost cells take part);
 3. the value is converted to A's variables, mass by sqrtG_A/sqrtG_B (3.26)
    and momentum by C = (sqrtG_A/sqrtG_B) J_A^-1 J_B (3.29), with J from
    (2.10)-(2.11);
 4. the ghost cell average is the Gauss quadrature (3.6) of the converted
    point values.

Because step 2 reads ghost cells, the ghost values are the fixed point of
this map; the oracle finds it by Jacobi sweeps from g = 0 (the paper's
iteration) until nothing changes, and ``dense_solve`` solves the same
fixed point as the linear system (7.10)-(7.12) for small grids.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import geometry as geo
from .weights import centred, gauss, weights_1d_f64


class GhostMap:
    """Geometry of all ghost GQPs of a grid and the fixed-point fill."""

    def __init__(self, n: int, k: int, radius: float, m: int | None = None):
        self.n, self.k = n, k
        self.r = r = (k - 1) // 2
        self.m = m = m or (k + 1) // 2
        self.P = P = n + 2 * r
        self.radius = radius
        self.delta = d = 0.5 * math.pi / n
        nodes, wts = gauss(m)
        cen = geo.cell_centres(n, r)        # centre of padded index ii, in units of Delta

        # ghost cells (panel, jj, ii) in padded indices
        jj, ii = np.meshgrid(np.arange(P), np.arange(P), indexing="ij")
        inner = (jj >= r) & (jj < r + n) & (ii >= r) & (ii < r + n)
        gj, gi = jj[~inner], ii[~inner]
        self.n_ghost_per_panel = gj.size
        gcell = []          # flat padded index of each ghost cell (panel*P*P + jj*P + ii)
        pt_ghost, pt_idx, pt_w, pt_s, pt_c = [], [], [], [], []
        for A in range(6):
            base = len(gcell)
            gcell.extend((A * P * P + gj * P + gi).tolist())
            # GQPs: per ghost cell, (h outer along y, g inner along x)
            xs = (cen[gi][:, None, None] + nodes[None, None, :]) * d      # (G, 1, m)
            ys = (cen[gj][:, None, None] + nodes[None, :, None]) * d      # (G, m, 1)
            xs, ys = np.broadcast_arrays(xs, ys)
            W = (wts[None, :, None] * wts[None, None, :]) * np.ones(xs.shape)
            gid = np.broadcast_to(np.arange(gj.size)[:, None, None], xs.shape) + base
            xs, ys, W, gid = xs.ravel(), ys.ravel(), W.ravel(), gid.ravel()
            XA, YA = np.tan(xs), np.tan(ys)
            v = geo.panel_xyz(A, XA, YA)
            best, second, tie = geo.owners(v)
            lam, th = geo.lonlat(v)
            JA = geo.j_paper(A, lam, th, radius)
            JAi = geo.inv2(JA)
            sgA = geo.sqrt_g(XA, YA, radius)
            for branch in (0, 1):
                if branch == 0:
                    sel = np.ones(xs.shape, bool)
                    Bs = best
                    fac = np.where(tie, 0.5, 1.0)
                else:
                    sel = tie
                    Bs = second
                    fac = np.full(xs.shape, 0.5)
                for B in range(6):
                    s = sel & (Bs == B)
                    if not s.any():
                        continue
                    assert B != A
                    XB, YB = geo.xyz_to_XY(B, v[s])
                    xb, yb = np.arctan(XB), np.arctan(YB)
                    ib = np.clip(np.floor(xb / d + n / 2.0), 0, n - 1).astype(np.int64)
                    jb = np.clip(np.floor(yb / d + n / 2.0), 0, n - 1).astype(np.int64)
                    xi = xb / d - (ib + 0.5 - n / 2.0)
                    eta = yb / d - (jb + 0.5 - n / 2.0)
                    wx = weights_1d_f64(centred(k), xi)          # (npt, k)
                    wy = weights_1d_f64(centred(k), eta)
                    w2 = wy[:, :, None] * wx[:, None, :]          # (npt, k, k)
                    offs = np.arange(k)
                    rows = jb[:, None] + offs[None, :]            # padded rows jb-r+r .. jb+r+r
                    cols = ib[:, None] + offs[None, :]
                    idx = B * P * P + rows[:, :, None] * P + cols[:, None, :]
                    JB = geo.j_paper(B, lam[s], th[s], radius)
                    sgB = geo.sqrt_g(XB, YB, radius)
                    ratio = sgA[s] / sgB
                    Cm = geo.mul2(tuple(c[s] for c in JAi), JB)
                    Cm = tuple(ratio * c for c in Cm)
                    q = W[s] * fac[s]
                    pt_ghost.append(gid[s])
                    pt_idx.append(idx.reshape(-1, k * k))
                    pt_w.append((w2 * q[:, None, None]).reshape(-1, k * k))
                    pt_s.append(ratio)
                    pt_c.append(np.stack(Cm, axis=-1))
        self.ghost_cells = torch.tensor(np.array(gcell), dtype=torch.int64)
        self.pt_ghost = torch.tensor(np.concatenate(pt_ghost), dtype=torch.int64)
        self.pt_idx = torch.tensor(np.concatenate(pt_idx), dtype=torch.int64)
        self.pt_w = torch.tensor(np.concatenate(pt_w))
        self.pt_s = torch.tensor(np.concatenate(pt_s))
        self.pt_c = torch.tensor(np.concatenate(pt_c))     # (npt, 4): C11 C12 C21 C22
        jjA, iiA = np.meshgrid(np.arange(r, r + n), np.arange(r, r + n), indexing="ij")
        self.interior = torch.tensor(
            np.concatenate([(A * P * P + jjA * P + iiA).ravel() for A in range(6)]), dtype=torch.int64)
        self.sweeps_used = None

    # ------------------------------------------------------------------
    def _assemble(self, q, g):
        P = self.P
        flat = torch.zeros(3, 6 * P * P, dtype=q.dtype)
        flat = flat.index_copy(1, self.interior, q.reshape(3, -1))
        flat = flat.index_copy(1, self.ghost_cells, g)
        return flat

    def _sweep(self, flat):
        vals = (flat[:, self.pt_idx] * self.pt_w).sum(-1)                    # (3, npt)
        mass = self.pt_s * vals[0]
        c = self.pt_c
        mu = c[:, 0] * vals[1] + c[:, 1] * vals[2]
        mv = c[:, 2] * vals[1] + c[:, 3] * vals[2]
        conv = torch.stack([mass, mu, mv])
        g = torch.zeros(3, self.ghost_cells.numel(), dtype=flat.dtype)
        return g.index_add(1, self.pt_ghost, conv)

    def fill(self, q: torch.Tensor, sweeps: int | None = None, max_sweeps: int = 200) -> torch.Tensor:
        """Padded state (3, 6, P, P) whose ghost cells hold the fixed point.

        q: interior cell averages (3, 6, n, n).  With ``sweeps`` given, exactly
        that many Jacobi sweeps from g = 0 (the paper fixes 10); otherwise
        sweep until the relative change of every variable is below 1e-15
        (the rounding floor is ~1e-16), then three more sweeps, and record
        the count in ``sweeps_used``.
        """
        g = torch.zeros(3, self.ghost_cells.numel(), dtype=q.dtype)
        count = 0
        extra = None
        while True:
            flat = self._assemble(q, g)
            g_new = self._sweep(flat)
            count += 1
            if sweeps is not None:
                g = g_new
                if count >= sweeps:
                    break
                continue
            with torch.no_grad():
                diff = (g_new - g).abs().amax(1)
                scale = g_new.abs().amax(1)
                small = bool(torch.all(diff <= 1e-15 * scale))
            g = g_new
            if small and extra is None:
                extra = 3
            if extra is not None:
                if extra == 0:
                    break
                extra -= 1
            if count >= max_sweeps:
                raise RuntimeError("ghost fixed point did not converge")
        self.sweeps_used = count
        return self._assemble(q, g).reshape(3, 6, self.P, self.P)

    # ------------------------------------------------------------------
    def dense_solve(self, q: torch.Tensor) -> torch.Tensor:
        """The same ghost values from the linear system (7.10)-(7.12).

        Builds, densely, the ghost update as g_new = L_q q + L_g g (the
        paper's A-bar, and C acting through B), then solves
        (I - L_g) g = L_q q directly.  For small grids only.
        """
        nq = 3 * 6 * self.n * self.n
        ng = 3 * self.ghost_cells.numel()
        Lq = torch.zeros(ng, nq, dtype=torch.float64)
        Lg = torch.zeros(ng, ng, dtype=torch.float64)
        zq = torch.zeros(3, 6, self.n, self.n, dtype=torch.float64)
        zg = torch.zeros(3, self.ghost_cells.numel(), dtype=torch.float64)
        for c in range(nq):
            e = zq.clone().reshape(-1)
            e[c] = 1.0
            Lq[:, c] = self._sweep(self._assemble(e.reshape(zq.shape), zg)).reshape(-1)
        for c in range(ng):
            e = zg.clone().reshape(-1)
            e[c] = 1.0
            Lg[:, c] = self._sweep(self._assemble(zq, e.reshape(zg.shape))).reshape(-1)
        g = torch.linalg.solve(torch.eye(ng, dtype=torch.float64) - Lg, Lq @ q.reshape(-1))
        return self._assemble(q, g.reshape(3, -1)).reshape(3, 6, self.P, self.P)
