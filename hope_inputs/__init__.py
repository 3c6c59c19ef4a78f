"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module describes the *physical* test states of the paper's experiments
(section 5) as pointwise fields on the unit sphere, plus seeded random draws
(perturbations, cotangents, cap centres, spherical-harmonic coefficients).
It holds none of the discretisation: no cubed-sphere panel map, no metric,
no reconstruction, flux or quadrature.  Each consumer projects these fields
onto its own cell averages with its own geometry code.

A field is a callable ``f(p) -> (phi, us, vs)`` where ``p`` is an array of
unit vectors of shape (..., 3), ``phi`` is geopotential (m^2/s^2) and
(us, vs) are the zonal and meridional winds (m/s).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Physical constants of the synthetic workloads.  The paper's case-2 radius is
# 6371220 m (section 5.1); the workloads use 6.371e6 m, kept as a parameter.
EARTH_RADIUS = 6.371e6
PAPER_RADIUS = 6371220.0
GRAVITY = 9.80616
OMEGA = 7.292e-5
DAY = 86400.0


def lonlat(p: np.ndarray):
    """Longitude and latitude (radians) of unit vectors p (..., 3)."""
    lam = np.arctan2(p[..., 1], p[..., 0])
    th = np.arcsin(np.clip(p[..., 2], -1.0, 1.0))
    return lam, th


# --------------------------------------------------------------------------
# Case 2 of the Williamson suite: steady geostrophic flow, eqs (5.1)-(5.3).
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class BalancedFlow:
    """Steady zonal geostrophic flow about an axis tilted by ``alpha``.

    Eqs (5.1)-(5.3): phi = phi0 - (a*Omega*u0 + u0^2/2) * s^2 with
    s = -cos(lam)cos(th)sin(alpha) + sin(th)cos(alpha), and the winds
    us = u0 (cos th cos alpha + cos lam sin th sin alpha),
    vs = -u0 sin lam sin alpha.  u0 = 2*pi*a / 12 days, phi0 = 2.94e4.
    The flow is balanced only when the Coriolis parameter uses the same
    tilted axis, f = 2*Omega*s.
    """

    alpha: float = 0.0
    radius: float = EARTH_RADIUS
    omega: float = OMEGA
    phi0: float = 2.94e4

    @property
    def u0(self) -> float:
        return 2.0 * math.pi * self.radius / (12.0 * DAY)

    def __call__(self, p):
        lam, th = lonlat(p)
        ca, sa = math.cos(self.alpha), math.sin(self.alpha)
        s = -np.cos(lam) * np.cos(th) * sa + np.sin(th) * ca
        u0 = self.u0
        phi = self.phi0 - (self.radius * self.omega * u0 + 0.5 * u0 * u0) * s * s
        us = u0 * (np.cos(th) * ca + np.cos(lam) * np.sin(th) * sa)
        vs = -u0 * np.sin(lam) * sa
        return phi, us, vs


# --------------------------------------------------------------------------
# Seeded smooth random field: real spherical harmonics up to degree lmax.
# --------------------------------------------------------------------------
def _real_sh_sum(p: np.ndarray, coef: np.ndarray, lmax: int) -> np.ndarray:
    """sum_{l,m} coef[l, m+lmax] * Y_lm(p) with orthonormal real harmonics.

    Associated Legendre functions by the standard stable recurrence on
    fully normalised P_l^m; cos(m lam)/sin(m lam) by angle addition.
    """
    lam, th = lonlat(p)
    x = np.sin(th)          # cos(colatitude)
    y = np.cos(th)          # sin(colatitude)
    out = np.zeros(x.shape)
    # normalised P_m^m
    pmm = np.full(x.shape, 1.0 / math.sqrt(4.0 * math.pi))
    cm = np.cos(lam)
    sm = np.sin(lam)
    cos_m = np.ones(x.shape)
    sin_m = np.zeros(x.shape)
    for m in range(0, lmax + 1):
        if m > 0:
            pmm = -math.sqrt((2.0 * m + 1.0) / (2.0 * m)) * y * pmm
            cos_m, sin_m = cos_m * cm - sin_m * sm, sin_m * cm + cos_m * sm
        plm_2 = None
        plm_1 = pmm
        for l in range(m, lmax + 1):
            if l == m:
                plm = pmm
            elif l == m + 1:
                plm = math.sqrt(2.0 * m + 3.0) * x * pmm
            else:
                a = math.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
                b = math.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
                plm = a * (x * plm_1 - b * plm_2)
            if l > m:
                plm_2, plm_1 = plm_1, plm
            if l >= 1:
                if m == 0:
                    out += coef[l, lmax] * plm
                else:
                    out += coef[l, lmax + m] * math.sqrt(2.0) * plm * cos_m
                    out += coef[l, lmax - m] * math.sqrt(2.0) * plm * sin_m
    return out


def fibonacci_sphere(n: int) -> np.ndarray:
    i = np.arange(n) + 0.5
    z = 1.0 - 2.0 * i / n
    r = np.sqrt(1.0 - z * z)
    phi = math.pi * (3.0 - math.sqrt(5.0)) * i
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=-1)


@dataclass
class SmoothRandomField:
    """S(p) = sum of real harmonics, degrees 1..lmax, coefficients
    N(0,1)/(l+1) drawn from ``seed``, scaled so that max |S| = 1 on a fixed
    20,000-point Fibonacci sampling of the sphere."""

    seed: int
    lmax: int = 20

    def __post_init__(self):
        rng = np.random.default_rng(self.seed)
        L = self.lmax
        coef = rng.standard_normal((L + 1, 2 * L + 1))
        for l in range(L + 1):
            coef[l] /= (l + 1.0)
            for mm in range(-L, L + 1):
                if abs(mm) > l:
                    coef[l, mm + L] = 0.0
        self.coef = coef
        s = _real_sh_sum(fibonacci_sphere(20000), coef, L)
        self.scale = 1.0 / float(np.max(np.abs(s)))

    def __call__(self, p):
        return self.scale * _real_sh_sum(p, self.coef, self.lmax)


def random_unit_vector(rng: np.random.Generator) -> np.ndarray:
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


def cap_indicator(p: np.ndarray, centre: np.ndarray, radius_frac: float) -> np.ndarray:
    """1 inside the spherical cap of great-circle radius radius_frac*a."""
    cosd = np.clip(p @ centre, -1.0, 1.0)
    return (np.arccos(cosd) < radius_frac).astype(np.float64)


@dataclass
class RestingLayer:
    """Resting layer h = h0 (+ cap jump dh inside a cap) (+ pert * h0 * S).

    The dam-break-like state (cap on) and the smooth random state (cap off).
    """

    seed: int
    h0: float = 1000.0
    cap_dh: float = 1000.0
    cap_radius: float = 0.2      # fraction of the radius (great-circle angle)
    with_cap: bool = True
    pert: float = 0.01
    lmax: int = 20
    gravity: float = GRAVITY

    def __post_init__(self):
        rng = np.random.default_rng(self.seed)
        self.centre = random_unit_vector(rng)
        self.sh = SmoothRandomField(seed=int(rng.integers(0, 2**31 - 1)), lmax=self.lmax)

    def __call__(self, p):
        h = np.full(p.shape[:-1], self.h0)
        if self.with_cap:
            h = h + self.cap_dh * cap_indicator(p, self.centre, self.cap_radius)
        if self.pert:
            h = h + self.pert * self.h0 * self.sh(p)
        z = np.zeros(p.shape[:-1])
        return self.gravity * h, z, z.copy()


@dataclass
class BalancedFlowWithCap:
    """Ensemble-member state: tilted balanced flow plus a cap height jump."""

    seed: int
    radius: float = EARTH_RADIUS
    gravity: float = GRAVITY
    omega: float = OMEGA

    def __post_init__(self):
        rng = np.random.default_rng(self.seed)
        self.alpha = float(rng.uniform(0.0, math.pi / 2))
        self.flow = BalancedFlow(alpha=self.alpha, radius=self.radius, omega=self.omega)
        h0 = self.flow.phi0 / self.gravity
        self.dh = float(rng.uniform(0.05, 0.2)) * h0
        self.cap_radius = float(rng.uniform(0.1, 0.3))
        self.centre = random_unit_vector(rng)

    def __call__(self, p):
        phi, us, vs = self.flow(p)
        phi = phi + self.gravity * self.dh * cap_indicator(p, self.centre, self.cap_radius)
        return phi, us, vs


def draw_tilt(seed: int) -> float:
    """Rotation-axis tilt alpha ~ U[0, pi/2]."""
    return float(np.random.default_rng(seed).uniform(0.0, math.pi / 2))


def normal_array(seed: int, shape) -> np.ndarray:
    """Standard-normal FP64 array (perturbations zeta, cotangents w)."""
    return np.random.default_rng(seed).standard_normal(shape)


def uniform_array(seed: int, shape, lo=-1.0, hi=1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, shape)
