"""Test workloads: seeded synthetic states with the shapes of the paper's
experiments (section 5), built with the oracle's projection of the shared
physical fields.  Used by the GPU parity tests and the smoke check."""
from __future__ import annotations

import math

import numpy as np
import torch

import hope_inputs as hi
from oracle.ic import cell_average
from oracle.rhs import Grid as OracleGrid
from oracle.rhs import Params

A = hi.EARTH_RADIUS


def balanced(n, seed=0, nq=4):
    alpha = hi.draw_tilt(seed)
    return alpha, cell_average(hi.BalancedFlow(alpha=alpha, radius=A), n, A, nq=nq)


def dam_break(n, seed=0, nq=4):
    return 0.0, cell_average(hi.RestingLayer(seed=seed), n, A, nq=nq)


def smooth_random(n, seed=0, nq=4):
    return 0.0, cell_average(hi.RestingLayer(seed=seed, with_cap=False), n, A, nq=nq)


def member(n, seed=0, nq=4):
    f = hi.BalancedFlowWithCap(seed=seed)
    return f.alpha, cell_average(f, n, A, nq=nq)


def perturbed_balanced(n, seed=0, nq=4):
    alpha, q = balanced(n, seed, nq)
    zeta = torch.tensor(hi.normal_array(seed + 1000, tuple(q.shape)))
    return alpha, q * (1.0 + 1e-3 * zeta)


def perturbed_member(n, seed=0, nq=4):
    """A member state with 0.1 % multiplicative noise.  The balanced flow is
    mirror-symmetric about the plane through the tilted rotation axis, and on
    that plane pairs of WENO smoothness indicators tie exactly, which puts
    the kink of |beta_a - beta_b| at the evaluation point: the derivative
    does not exist there and a gradient comparison is meaningless.  The noise
    moves every state off such ties."""
    alpha, q = member(n, seed, nq)
    zeta = torch.tensor(hi.normal_array(seed + 2000, tuple(q.shape)))
    return alpha, q * (1.0 + 1e-3 * zeta)


def smooth_cell_field(n, seed) -> torch.Tensor:
    """(6, n, n) values at the cell centres of a seeded smooth random field
    (spherical harmonics up to degree 20, max |.| = 1)."""
    from oracle import geometry as geo
    f = hi.SmoothRandomField(seed=seed)
    X = np.tan(geo.cell_centres(n, 0) * (0.5 * math.pi / n))
    return torch.tensor(np.stack([f(geo.panel_xyz(p, X[None, :], X[:, None])) for p in range(6)]))


def smooth_perturbed_balanced(n, seed=0, nq=4):
    """A balanced flow times (1 + 1 % smooth random field): smooth, moving,
    and without the mirror symmetry of the balanced flow."""
    alpha, q = balanced(n, seed, nq)
    return alpha, q * (1.0 + 1e-2 * smooth_cell_field(n, seed + 3000))


def rossby_haurwitz(n, seed=0, nq=4):
    """The wavenumber-4 Rossby-Haurwitz wave of (5.10)-(5.12) (no seeded
    part; seed unused), at the radius the other states use."""
    return 0.0, cell_average(hi.RossbyHaurwitz(radius=A), n, A, nq=nq)


STATES = {"rossby_haurwitz": rossby_haurwitz, "balanced": balanced, "dam_break": dam_break, "smooth_random": smooth_random, "member": member,
          "perturbed_balanced": perturbed_balanced, "perturbed_member": perturbed_member,
          "smooth_perturbed_balanced": smooth_perturbed_balanced}


def oracle_grid(n, order, scheme, alpha):
    return OracleGrid(n, order, scheme, Params(alpha=alpha))


def to_padded(q: torch.Tensor, r: int, device="cuda") -> torch.Tensor:
    n = q.shape[-1]
    P = n + 2 * r
    out = torch.zeros(3, 6, P, P, dtype=torch.float64)
    out[:, :, r:r + n, r:r + n] = q
    return out.to(device).contiguous()


def rel_err(a: torch.Tensor, b: torch.Tensor):
    """Per variable: max |a - b| / max |b| (L-infinity relative over all cells)."""
    a = a.detach().double().cpu()
    b = b.detach().double().cpu()
    return [float((a[v] - b[v]).abs().max() / b[v].abs().max().clamp_min(1e-300)) for v in range(3)]


def cfl_dt(q: torch.Tensor, radius=A, cfl=0.5):
    """dt = cfl * Delta / max(|u^i| + sqrt(phi) sqrt(G^ii)) over cells (harness
    rule; the method itself takes dt as given)."""
    n = q.shape[-1]
    d = 0.5 * math.pi / n
    x = (np.arange(n) + 0.5 - n / 2) * d
    X = np.tan(x)[None, :]
    Y = np.tan(x)[:, None]
    d2 = 1 + X * X + Y * Y
    sg = radius ** 2 * (1 + X * X) * (1 + Y * Y) / d2 ** 1.5
    qn = q.numpy()
    phi = qn[0] / sg
    u = qn[1] / qn[0]
    v = qn[2] / qn[0]
    g11 = d2 / (radius ** 2 * (1 + X * X))
    g22 = d2 / (radius ** 2 * (1 + Y * Y))
    s = np.maximum(np.abs(u) + np.sqrt(phi * g11), np.abs(v) + np.sqrt(phi * g22))
    return cfl * d / float(s.max())
