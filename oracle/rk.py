"""Three-stage explicit Runge-Kutta time stepping (section 3.5).
Test infrastructure only.

``ssp_rk3`` is the strong-stability-preserving three-stage scheme of Shu and
Osher used by the workloads; ``ws_rk3`` is the scheme the paper prints,
(3.39)-(3.41), with the second stage read as q** = q^n + dt/2 L(q*) (the
printed q* + dt/2 L(q*) is not third order).  Both have the stability
polynomial 1 + z + z^2/2 + z^3/6 on linear problems.
"""
from __future__ import annotations


def ssp_rk3(L, q, dt):
    q1 = q + dt * L(q)
    q2 = 0.75 * q + 0.25 * (q1 + dt * L(q1))
    return q / 3.0 + (2.0 / 3.0) * (q2 + dt * L(q2))


def ws_rk3(L, q, dt):
    q1 = q + (dt / 3.0) * L(q)          # (3.39)
    q2 = q + (dt / 2.0) * L(q1)         # (3.40), read with q^n
    return q + dt * L(q2)               # (3.41)
