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


# --------------------------------------------------------------------------
# Rossby-Haurwitz wave with wavenumber R = 4, eqs (5.9)-(5.15).
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class RossbyHaurwitz:
    """phi = phi0 + a^2 [A(th) + B(th) cos(R lam) + C(th) cos(2 R lam)] (5.10),
    us = a w cos th + a K cos^(R-1) th (R sin^2 th - cos^2 th) cos(R lam) (5.11),
    vs = -a K R cos^(R-1) th sin th sin(R lam) (5.12), with A, B, C of
    (5.13)-(5.15), K = w = 7.848e-6 1/s, h0 = 8000 m.  ``shift`` rotates
    the pattern eastwards by that many radians (the pattern at time t is,
    for the barotropic vorticity equation, the initial one shifted by c t
    with the angular phase speed c of (5.9))."""

    radius: float = PAPER_RADIUS
    omega: float = OMEGA
    w: float = 7.848e-6
    wavenumber: int = 4
    h0: float = 8000.0
    gravity: float = GRAVITY
    shift: float = 0.0

    @property
    def phase_speed(self) -> float:
        """Angular phase speed c of (5.9), rad/s."""
        R = self.wavenumber
        return (R * (R + 3) * self.w - 2.0 * self.omega) / ((R + 1) * (R + 2))

    def __call__(self, p):
        lam, th = lonlat(p)
        lam = lam - self.shift
        R, w, K, a, Om = self.wavenumber, self.w, self.w, self.radius, self.omega
        c, s = np.cos(th), np.sin(th)
        c2 = c * c
        # cos^(2R) th times the bracket of (5.13), with its cos^-2 th term folded
        # into the power so that the poles need no division
        A = 0.5 * w * (2.0 * Om + w) * c2 + 0.25 * K * K * (
            (R + 1) * c ** (2 * R + 2) + (2.0 * R * R - R - 2.0) * c ** (2 * R) - 2.0 * R * R * c ** (2 * R - 2))
        B = 2.0 * (Om + w) * K / ((R + 1) * (R + 2)) * c ** R * (R * R + 2 * R + 2 - (R + 1) ** 2 * c2)
        C = 0.25 * K * K * c ** (2 * R) * ((R + 1) * c2 - R - 2.0)
        phi = self.gravity * self.h0 + a * a * (A + B * np.cos(R * lam) + C * np.cos(2 * R * lam))
        us = a * w * c + a * K * c ** (R - 1) * (R * s * s - c2) * np.cos(R * lam)
        vs = -a * K * R * c ** (R - 1) * s * np.sin(R * lam)
        return phi, us, vs


# --------------------------------------------------------------------------
# Bottom topography (section 2, (2.13)-(2.14)) and the states over it.  A
# surface is a callable phis(p) -> surface geopotential g h_s (m^2/s^2).  A
# field over topography returns the layer's own geopotential phi = g h
# (depth), so that phi + phis is the total (free-surface) geopotential.
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class ConeMountain:
    """The isolated mountain of section 5.2, (5.8): h_s = h_s0 (1 - r/R) with
    r = sqrt(min(R^2, (lam - lam_c)^2 + (th - th_c)^2)), h_s0 = 2000 m,
    R = pi/9, (lam_c, th_c) = (3 pi/2, pi/6); longitudes in [0, 2 pi).  Its
    slope is discontinuous at the peak and along the rim."""

    hs0: float = 2000.0
    R: float = math.pi / 9
    lam_c: float = 1.5 * math.pi
    th_c: float = math.pi / 6
    gravity: float = GRAVITY

    def __call__(self, p):
        lam, th = lonlat(p)
        lam = np.mod(lam, 2.0 * math.pi)
        r = np.sqrt(np.minimum(self.R ** 2, (lam - self.lam_c) ** 2 + (th - self.th_c) ** 2))
        return self.gravity * self.hs0 * (1.0 - r / self.R)


@dataclass(frozen=True)
class MountainFlow:
    """Initial state of section 5.2: the zonal flow of (5.1)-(5.3) with
    h0 = 5960 m and u0 = 20 m/s (untilted), whose free surface follows the
    balanced profile, over the cone: depth phi = phi_total - phis."""

    radius: float = PAPER_RADIUS
    omega: float = OMEGA
    gravity: float = GRAVITY
    h0: float = 5960.0
    u0: float = 20.0

    @property
    def surface(self):
        return ConeMountain(gravity=self.gravity)

    def __call__(self, p):
        lam, th = lonlat(p)
        s = np.sin(th)
        phit = self.gravity * self.h0 - (self.radius * self.omega * self.u0 + 0.5 * self.u0 ** 2) * s * s
        us = self.u0 * np.cos(th)
        return phit - self.surface(p), us, np.zeros_like(us)


@dataclass(frozen=True)
class LakeAtRest:
    """Fluid at rest with a flat free surface over a surface: depth
    phi = phit0 - phis, no wind.  The exact state whose preservation is the
    "C-property" of section 2."""

    surface: object
    phit0: float = GRAVITY * 5960.0

    def __call__(self, p):
        z = np.zeros(p.shape[:-1])
        return self.phit0 - self.surface(p), z, z.copy()


@dataclass(frozen=True)
class AxisRidge:
    """A smooth ridge that is constant along the circles about an axis tilted
    by alpha (the flow lines of the tilted balanced flow):
    phis = g h_r exp(-((s - s0)/w)^2), s = -cos(lam)cos(th)sin(alpha) + sin(th)cos(alpha)."""

    alpha: float = 0.0
    h_r: float = 400.0
    s0: float = 0.3
    width: float = 0.4
    gravity: float = GRAVITY

    def __call__(self, p):
        lam, th = lonlat(p)
        ca, sa = math.cos(self.alpha), math.sin(self.alpha)
        s = -np.cos(lam) * np.cos(th) * sa + np.sin(th) * ca
        return self.gravity * self.h_r * np.exp(-((s - self.s0) / self.width) ** 2)


@dataclass(frozen=True)
class BalancedFlowOverRidge:
    """An exact steady state with topography: the tilted balanced flow of
    (5.1)-(5.3) whose free surface is the balanced profile, over an AxisRidge
    about the same axis, depth phi = phi_balanced - phis.  The ridge is
    constant along the (non-divergent) flow lines, so the mass flux divergence
    is unchanged, and the momentum balance involves only the total
    geopotential (2.13)-(2.14), which is that of the balanced flow."""

    alpha: float = 0.0
    radius: float = EARTH_RADIUS
    omega: float = OMEGA
    gravity: float = GRAVITY

    @property
    def surface(self):
        return AxisRidge(alpha=self.alpha, gravity=self.gravity)

    def __call__(self, p):
        phi, us, vs = BalancedFlow(alpha=self.alpha, radius=self.radius, omega=self.omega)(p)
        return phi - self.surface(p), us, vs
