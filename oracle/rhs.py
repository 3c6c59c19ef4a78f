"""Right-hand side of the cubed-sphere shallow-water finite-volume core,
written step by step from sections 2-3 of the paper.  Test infrastructure only.

State: cell averages (over dx dy in angular coordinates) of
q = (sqrtG phi, sqrtG phi u, sqrtG phi v) (2.15)-(2.16), shape (3, 6, n, n),
index [variable, panel, j (y), i (x)].

With bottom topography (section 2, (2.13)-(2.14)) the reconstruction
variables are (sqrtG phi_t, sqrtG phi u, sqrtG phi v), phi_t = phi + phi_s:
the cell averages of sqrtG phi_s are added to the mass before the ghost fill
and the reconstruction, and subtracted again, as point values, at every edge
and cell Gauss point; the LMARS pressure uses phi_t* = phi* + phi_s and the
sources gain psi_B = sqrtG phi_s G^ij d(phi_t)/dx^j.

Per evaluation (section 3):
  1. ghost cells by the fixed-point interpolation (section 3.3.1)     ghost.py
  2. reconstruction at the edge Gauss points (EQPs) and cell Gauss points
     (CQPs) of every cell: TPP (3.7)-(3.15) or genuine 2D WENO (3.16)-(3.25)
  3. at panel edges the outside state is the neighbour panel's own trace,
     converted into this panel's variables (3.26)-(3.29)
  4. LMARS flux at every EQP (3.30)-(3.38)
  5. Gauss quadrature of the edge fluxes (3.5) and of the sources at the CQPs
     (3.6); sources are the metric term (2.2) and Coriolis term (2.3)
  6. tendency (3.1)
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import geometry as geo
from .ghost import GhostMap
from .weights import (axis_derivative_weights, axis_weights, centred,
                      derivative_gram, gauss, split_weights, substencil_offsets,
                      substencil_poly_1d, weno_linear_weights)


@dataclass
class Params:
    radius: float = 6.371e6
    gravity: float = 9.80616
    omega: float = 7.292e-5
    alpha: float = 0.0          # tilt of the rotation axis (radians)
    weno_eps: float = 1e-12
    split_theta: float = 3.0
    surface: object = None      # phis(p) -> surface geopotential g h_s at unit vectors p, or None


def _t(a):
    return torch.as_tensor(np.asarray(a), dtype=torch.float64)


def apply_stencil(qpad, n, wy, wx, y0, x0):
    """sum_{b,a} wy[b] wx[a] qpad[..., y0+b+j, x0+a+i] for the n x n interior
    cells (i, j): the TPP reconstruction (3.14) with the tensor-product weights."""
    out = 0.0
    for b in range(wy.shape[0]):
        for a in range(wx.shape[0]):
            out = out + wy[b] * wx[a] * qpad[..., y0 + b:y0 + b + n, x0 + a:x0 + a + n]
    return out


class WenoTables:
    """Genuine 2D WENO of order n (section 3.2): sub-stencil weights, linear
    weights gamma and their split, smoothness-indicator forms."""

    def __init__(self, order: int, m: int, theta: float = 3.0, eps: float = 1e-12):
        self.n_order = order
        self.m = m
        self.l = (order + 1) // 2
        self.r = (order - 1) // 2
        self.eps = eps
        self.subs = substencil_offsets(order)
        self.ws = {s: _t(axis_weights(tuple(range(s, s + self.l)), m)) for s in range(-(self.l - 1), 1)}
        gam, _ = weno_linear_weights(order, m)
        self.gamma = _t(gam)
        gp, gm, sp, sm = split_weights(gam, theta)
        self.gp, self.gm, self.sp, self.sm = _t(gp), _t(gm), _t(sp), _t(sm)
        self.poly = {s: _t([[float(v) for v in row] for row in substencil_poly_1d(self.l, s)])
                     for s in range(-(self.l - 1), 1)}
        self.K = [_t([[float(v) for v in row] for row in Ka]) for Ka in derivative_gram(self.l)]

    def beta(self, qpad, n):
        """Smoothness indicator of every sub-stencil polynomial over the
        target cell: sum over derivative orders (a, b) != (0, 0), a, b < l, of
        the integral of the squared derivative (reading of (3.25))."""
        l, r = self.l, self.r
        betas = []
        for (sx, sy) in self.subs:
            # coefficient matrix Cf[beta, alpha] of p_j = sum Cf x^alpha y^beta
            My, Mx = self.poly[sy], self.poly[sx]
            cells = torch.stack([torch.stack([qpad[..., r + sy + b:r + sy + b + n, r + sx + a:r + sx + a + n]
                                              for a in range(l)], -1) for b in range(l)], -2)   # (..., l_b, l_a)
            Cf = torch.einsum("Bb,...ba,Aa->...BA", My, cells, Mx)
            beta = 0.0
            for a in range(l):
                for b in range(l):
                    if a == 0 and b == 0:
                        continue
                    tmp = torch.einsum("BC,...CD,DA->...BA", self.K[b], Cf, self.K[a])
                    beta = beta + (Cf * tmp).sum((-1, -2))
            betas.append(beta)
        return torch.stack(betas)        # (s, ..., n, n)

    @staticmethod
    def tau(beta):
        """(3.24): 2/(s(s+1)) times the sum over pairs of |beta_psi - beta_eta|."""
        s = beta.shape[0]
        t = 0.0
        for i in range(s):
            for j in range(i + 1, s):
                t = t + (beta[i] - beta[j]).abs()
        return t * (2.0 / (s * (s + 1)))

    def value(self, qpad, n, ax, ay, pt, beta, tau):
        """WENO-Z value at one point of every cell, (3.20)-(3.23) with the
        split combination sigma+ sum w+ p - sigma- sum w- p."""
        r = self.r
        ps = torch.stack([apply_stencil(qpad, n, self.ws[sy][ay], self.ws[sx][ax], r + sy, r + sx)
                          for (sx, sy) in self.subs])
        kappa = 1.0 + tau / (beta + self.eps)
        shape = (-1,) + (1,) * (ps.dim() - 1)
        ap = self.gp[pt].reshape(shape) * kappa
        am = self.gm[pt].reshape(shape) * kappa
        wp = ap / ap.sum(0)
        wm = am / am.sum(0)
        return self.sp[pt] * (wp * ps).sum(0) - self.sm[pt] * (wm * ps).sum(0)


class Grid:

    """Everything the oracle precomputes for one (n, order, scheme)."""

    def __init__(self, n: int, order: int, scheme: str = "tpp", params: Params | None = None,
                 m: int | None = None):
        assert order % 2 == 1 and scheme in ("tpp", "weno")
        self.n, self.k, self.scheme = n, order, scheme
        self.p = params or Params()
        self.r = (order - 1) // 2
        self.m = m or (order + 1) // 2
        self.P = n + 2 * self.r
        self.delta = 0.5 * math.pi / n
        self.ghost = GhostMap(n, order, self.p.radius, self.m)
        nodes, wts = gauss(self.m)
        self.nodes, self.gw = nodes, _t(wts)
        # axis weights of the centred stencil: rows [-1/2, +1/2, g_1..g_m]
        self.wc = _t(axis_weights(centred(order), self.m))
        if scheme == "weno":
            self.weno = WenoTables(order, self.m, self.p.split_theta, self.p.weno_eps)
        self._metric()
        self._boundary_maps()
        self.topo = self.p.surface is not None
        if self.topo:
            self._topography()

    # ------------------------------------------------------------------
    # metric at the function points
    # ------------------------------------------------------------------
    def _metric(self):
        n, d = self.n, self.delta
        cen = geo.cell_centres(n, 0)                       # (n,)
        e = (np.arange(n + 1) - n / 2.0) * d               # edge coordinates
        Xe = np.tan(e)
        Xe[0], Xe[-1] = -1.0, 1.0                          # panel edges exactly at X = -+1
        Xg = np.tan((cen[:, None] + self.nodes[None, :]) * d)   # (n, m): cell i, node h
        self.Xe, self.Xg = Xe, Xg

    def _boundary_maps(self):
        """For each panel side, where the neighbour's trace lives and the
        conversion into this panel's variables (3.26)-(3.29)."""
        n, m, d, a = self.n, self.m, self.delta, self.p.radius
        self.bmap = {}
        node_list = self.nodes
        for A in range(6):
            for side in range(4):                     # 0 left (x=-pi/4), 1 right, 2 bottom, 3 top
                t = np.tan((geo.cell_centres(n, 0)[:, None] + node_list[None, :]) * d)   # (n, m)
                sgn = -1.0 if side in (0, 2) else 1.0
                if side < 2:
                    XA, YA = np.full(t.shape, sgn), t
                    Xo, Yo = np.tan(sgn * (0.25 * math.pi + 0.5 * d)), np.zeros(1)
                else:
                    XA, YA = t, np.full(t.shape, sgn)
                    Xo, Yo = np.zeros(1), np.tan(sgn * (0.25 * math.pi + 0.5 * d))
                B = int(geo.owners(geo.panel_xyz(A, Xo, Yo))[0][0])
                v = geo.panel_xyz(A, XA, YA)
                XB, YB = geo.xyz_to_XY(B, v)
                if np.all(np.abs(np.abs(XB) - 1) < 1e-9):
                    bside = 0 if XB.mean() < 0 else 1
                    along = np.arctan(YB)
                else:
                    assert np.all(np.abs(np.abs(YB) - 1) < 1e-9)
                    bside = 2 if YB.mean() < 0 else 3
                    along = np.arctan(XB)
                idx = np.clip(np.floor(along / d + n / 2.0), 0, n - 1).astype(np.int64)
                loc = along / d - (idx + 0.5 - n / 2.0)
                hb = np.abs(loc[..., None] - node_list[None, None, :]).argmin(-1)
                assert np.abs(loc - node_list[hb]).max() < 1e-8
                lam, th = geo.lonlat(v)
                JA = geo.j_paper(A, lam, th, a)
                JB = geo.j_paper(B, lam, th, a)
                ratio = geo.sqrt_g(XA, YA, a) / geo.sqrt_g(XB, YB, a)
                Cm = geo.mul2(geo.inv2(JA), JB)
                Cm = np.stack([ratio * c for c in Cm], -1)          # (n, m, 4)
                self.bmap[(A, side)] = (B, bside, torch.as_tensor(idx), torch.as_tensor(hb),
                                        _t(ratio), _t(Cm))

    def _topography(self, nq: int = 4):
        """Surface geopotential phi_s (section 2): cell averages of
        sqrtG phi_s (nq x nq Gauss rule per cell), which turn the layer's
        mass into the reconstruction variable sqrtG phi_t of (2.13), and
        sqrtG phi_s at every edge point (x edges (6, n, n+1), y edges
        (6, n+1, n), per Gauss node) and cell point ((6, n, n) per node pair).
        Also the derivative weights of the centred stencil, d/dxi of (3.14),
        for d(phi_t)/dx^j in psi_B (2.14)."""
        n, m, d, a = self.n, self.m, self.delta, self.p.radius
        f = self.p.surface
        nodes, wts = gauss(nq)
        xs = (geo.cell_centres(n, 0)[:, None] + nodes[None, :]) * d
        X, Y = np.broadcast_arrays(np.tan(xs)[None, None, :, :], np.tan(xs)[:, :, None, None])
        w = wts[None, :, None, None] * wts[None, None, None, :]
        sg = geo.sqrt_g(X, Y, a)
        self.sbar = _t(np.stack([(sg * f(geo.panel_xyz(p, X, Y)) * w).sum(axis=(1, 3)) for p in range(6)]))

        def s_at(X, Y):
            X, Y = np.broadcast_arrays(X, Y)
            return _t(np.stack([geo.sqrt_g(X, Y, a) * f(geo.panel_xyz(p, X, Y)) for p in range(6)]))

        self.s_xe = [s_at(self.Xe[None, :], self.Xg[:, h][:, None]) for h in range(m)]
        self.s_ye = [s_at(self.Xg[:, h][None, :], self.Xe[:, None]) for h in range(m)]
        self.s_cq = [[s_at(self.Xg[:, h][None, :], self.Xg[:, v][:, None]) for h in range(m)] for v in range(m)]
        self.wd = _t(axis_derivative_weights(centred(self.k), m))

    # ------------------------------------------------------------------
    # reconstruction
    # ------------------------------------------------------------------
    def _tpp(self, qpad, ax, ay):
        return apply_stencil(qpad, self.n, self.wc[ay], self.wc[ax], 0, 0)

    def reconstruct(self, qpad):
        """Values at all EQPs and CQPs of every interior cell.

        Returns xe[side][h], ye[side][h] and cq[v][h], each (3, 6, n, n):
        xe at (xi, eta) = (-+1/2, g_h); ye at (g_h, -+1/2); cq at (g_h, g_v).
        """
        m = self.m
        if self.scheme == "tpp":
            f = lambda ax, ay, pt: self._tpp(qpad, ax, ay)
        else:
            wt = self.weno
            beta = wt.beta(qpad, self.n)
            tau = wt.tau(beta)
            f = lambda ax, ay, pt: wt.value(qpad, self.n, ax, ay, pt, beta, tau)
        # point numbering follows weights.cell_points
        xe = [[f(side, 2 + h, side * m + h) for h in range(m)] for side in range(2)]
        ye = [[f(2 + h, side, 2 * m + side * m + h) for h in range(m)] for side in range(2)]
        cq = [[f(2 + h, 2 + v, 4 * m + v * m + h) for h in range(m)] for v in range(m)]
        return xe, ye, cq

    # ------------------------------------------------------------------
    # Riemann solver (3.30)-(3.38)
    # ------------------------------------------------------------------
    def lmars(self, qL, qR, X, Y, direction, phis=None):
        """phis: surface geopotential at the points (topography): the
        pressure (3.38) then uses phi_t* = phi* + phis, with phi* of (3.33)
        from the layer's own phi on both sides."""
        a = self.p.radius
        sg = _t(geo.sqrt_g(X, Y, a))
        g11, g12, g22 = (_t(v) for v in geo.g_upper(X, Y, a))
        gii = g11 if direction == 1 else g22
        sq = torch.sqrt(gii)
        phiL, phiR = qL[0] / sg, qR[0] / sg
        vel = 1 if direction == 1 else 2
        upL = (qL[vel] / qL[0]) / sq                     # (3.31)
        upR = (qR[vel] / qR[0]) / sq
        c = 0.5 * (torch.sqrt(phiL) + torch.sqrt(phiR))  # (3.34)-(3.35)
        mstar = 0.5 * (upL + upR - (phiR - phiL) / c)    # (3.32)
        phistar = 0.5 * (phiL + phiR - c * (upR - upL))  # (3.33)
        mm = mstar * sq                                  # (3.36)
        F = 0.5 * (mm * (qL + qR) - mm.abs() * (qR - qL))   # (3.37), upwind term |m|
        if phis is not None:
            phistar = phistar + phis
        pres = 0.5 * sg * phistar * phistar                 # (3.38)
        if direction == 1:
            P = torch.stack([torch.zeros_like(pres), pres * g11, pres * g12])
        else:
            P = torch.stack([torch.zeros_like(pres), pres * g12, pres * g22])
        return F + P

    # ------------------------------------------------------------------
    def outside_traces(self, xe, ye):
        """Neighbour traces at the EQPs of each panel side, converted to this
        panel's variables.  Returns out[(A, side)] of shape (3, n, m)."""
        out = {}
        for (A, side), (B, bside, idx, hb, ratio, Cm) in self.bmap.items():
            if bside < 2:
                col = 0 if bside == 0 else self.n - 1
                S = torch.stack([xe[bside][h][:, B, :, col] for h in range(self.m)], -1)    # (3, n, m)
            else:
                row = 0 if bside == 2 else self.n - 1
                S = torch.stack([ye[bside - 2][h][:, B, row, :] for h in range(self.m)], -1)
            # B's trace at B's cell idx[t, h] and B's node hb[t, h]
            vals = S.reshape(3, -1)[:, (idx * self.m + hb).reshape(-1)].reshape(3, self.n, self.m)
            mass = ratio * vals[0]
            mu = Cm[..., 0] * vals[1] + Cm[..., 1] * vals[2]
            mv = Cm[..., 2] * vals[1] + Cm[..., 3] * vals[2]
            out[(A, side)] = torch.stack([mass, mu, mv])
        return out

    # ------------------------------------------------------------------
    def tendency(self, q: torch.Tensor, ghost_sweeps: int | None = None) -> torch.Tensor:
        """dq/dt of (3.1) for interior cell averages q (3, 6, n, n)."""
        n, m, d = self.n, self.m, self.delta
        qr = q
        if self.topo:
            # reconstruction variables (sqrtG phi_t, sqrtG phi u, sqrtG phi v) (2.13)
            qr = torch.cat([q[:1] + self.sbar, q[1:]])
        qpad = self.ghost.fill(qr, sweeps=ghost_sweeps)
        xe, ye, cq = self.reconstruct(qpad)
        outs = self.outside_traces(xe, ye)

        # ---- x-edges: edge e between cells e-1 and e, e = 0..n -------------
        Fbar = 0.0
        for h in range(m):
            left = xe[1][h]                    # right trace of each cell   (3, 6, n, n)
            right = xe[0][h]                   # left trace of each cell
            qL = torch.cat([torch.stack([outs[(A, 0)][:, :, h] for A in range(6)], 1)[..., None], left], -1)
            qR = torch.cat([right, torch.stack([outs[(A, 1)][:, :, h] for A in range(6)], 1)[..., None]], -1)
            X = self.Xe[None, :]                               # (1, n+1)
            Y = self.Xg[:, h][:, None]                         # (n, 1)
            X, Y = np.broadcast_arrays(X, Y)
            phis = None
            if self.topo:
                sp = self.s_xe[h]                              # sqrtG phi_s, same on both sides
                qL = torch.cat([qL[:1] - sp, qL[1:]])
                qR = torch.cat([qR[:1] - sp, qR[1:]])
                phis = sp / _t(geo.sqrt_g(X, Y, self.p.radius))
            F = self.lmars(qL, qR, X, Y, 1, phis)              # (3, 6, n, n+1)
            Fbar = Fbar + self.gw[h] * F
        # ---- y-edges ------------------------------------------------------
        Gbar = 0.0
        for h in range(m):
            below = ye[1][h]
            above = ye[0][h]
            qL = torch.cat([torch.stack([outs[(A, 2)][:, :, h] for A in range(6)], 1)[..., None, :], below], -2)
            qR = torch.cat([above, torch.stack([outs[(A, 3)][:, :, h] for A in range(6)], 1)[..., None, :]], -2)
            X = self.Xg[:, h][None, :]                         # (1, n) along i
            Y = self.Xe[:, None]                               # (n+1, 1)
            X, Y = np.broadcast_arrays(X, Y)
            phis = None
            if self.topo:
                sp = self.s_ye[h]
                qL = torch.cat([qL[:1] - sp, qL[1:]])
                qR = torch.cat([qR[:1] - sp, qR[1:]])
                phis = sp / _t(geo.sqrt_g(X, Y, self.p.radius))
            G = self.lmars(qL, qR, X, Y, 2, phis)              # (3, 6, n+1, n)
            Gbar = Gbar + self.gw[h] * G
        # ---- sources at the CQPs ------------------------------------------
        S = self.sources(cq, qpad)
        dq = -(Fbar[..., 1:] - Fbar[..., :-1]) / d - (Gbar[..., 1:, :] - Gbar[..., :-1, :]) / d + S
        return dq

    def sources(self, cq, qpad=None):
        """Cell average (3.6) of S = (0, psi_M + psi_C + psi_B) (2.2)-(2.3),
        (2.14).  With topography cq holds sqrtG phi_t at the cell points; the
        layer's sqrtG phi is that minus sqrtG phi_s, and psi_B takes
        d(phi_t)/dx^j from the derivative of the order-k polynomial of
        sqrtG phi_t on the centred stencil (the linear reconstruction, also
        under WENO): d/dx = (1/Delta) d/dxi, and
        d(phi_t)/dx = (d(sqrtG phi_t)/dx - phi_t d(sqrtG)/dx) / sqrtG with
        d(ln sqrtG)/dx = X (2Y^2 - X^2 - 1) / delta^2 from (2.8)."""
        n, m, a = self.n, self.m, self.p.radius
        Sbar1, Sbar2 = 0.0, 0.0
        for v in range(m):
            for h in range(m):
                X = self.Xg[:, h][None, :]   # (1, n)  cell i
                Y = self.Xg[:, v][:, None]   # (n, 1)  cell j
                X, Y = np.broadcast_arrays(X, Y)
                Q0, Q1, Q2 = cq[v][h][0], cq[v][h][1], cq[v][h][2]
                sg = _t(geo.sqrt_g(X, Y, a))
                g11, g12, g22 = (_t(t) for t in geo.g_upper(X, Y, a))
                Xt, Yt = _t(X), _t(Y)
                d2 = 1.0 + Xt * Xt + Yt * Yt
                psiB1, psiB2 = 0.0, 0.0
                if self.topo:
                    Tt = Q0                                     # sqrtG phi_t at the point
                    sp = self.s_cq[v][h]
                    Q0 = Tt - sp
                    Txi = apply_stencil(qpad[0], n, self.wc[2 + v], self.wd[2 + h], 0, 0)
                    Teta = apply_stencil(qpad[0], n, self.wd[2 + v], self.wc[2 + h], 0, 0)
                    dx = (Txi / self.delta - Tt * Xt * (2.0 * Yt * Yt - Xt * Xt - 1.0) / d2) / sg
                    dy = (Teta / self.delta - Tt * Yt * (2.0 * Xt * Xt - Yt * Yt - 1.0) / d2) / sg
                    psiB1 = sp * (g11 * dx + g12 * dy)          # (2.14)
                    psiB2 = sp * (g12 * dx + g22 * dy)
                phi = Q0 / sg
                u = Q1 / Q0
                vv = Q2 / Q0
                psiM1 = 2.0 * sg / d2 * (-Xt * Yt * Yt * phi * u * u + Yt * (1.0 + Yt * Yt) * phi * u * vv)
                psiM2 = 2.0 * sg / d2 * (Xt * (1.0 + Xt * Xt) * phi * u * vv - Xt * Xt * Yt * phi * vv * vv)
                fs = []
                for A in range(6):
                    pv = geo.panel_xyz(A, X, Y)
                    fs.append(_t(geo.coriolis_f(pv, self.p.omega, self.p.alpha)))
                f = torch.stack(fs)                      # (6, n, n)
                psiC1 = sg * f * (-g12 * Q1 + g11 * Q2)
                psiC2 = sg * f * (-g22 * Q1 + g12 * Q2)
                w = self.gw[h] * self.gw[v]
                Sbar1 = Sbar1 + w * (psiM1 + psiC1 + psiB1)
                Sbar2 = Sbar2 + w * (psiM2 + psiC2 + psiB2)
        return torch.stack([torch.zeros_like(Sbar1), Sbar1, Sbar2])
