"""Diagnostics: total mass and the error norms (5.4)-(5.7).
Test infrastructure only."""
from __future__ import annotations

import math

import numpy as np
import torch


def mass(q: torch.Tensor) -> torch.Tensor:
    """Integral of phi over the sphere: Delta^2 * sum of the cell averages of sqrtG phi."""
    n = q.shape[-1]
    d = 0.5 * math.pi / n
    return d * d * q[0].sum()


def error_norms(phi: np.ndarray, phi_ref: np.ndarray, sg_cell: np.ndarray):
    """(5.4)-(5.7) with absolute values: I(f) = sum sqrtG f over all cells."""
    I = lambda f: float((sg_cell * f).sum())
    l1 = I(np.abs(phi - phi_ref)) / I(np.abs(phi_ref))
    l2 = math.sqrt(I((phi - phi_ref) ** 2) / I(phi_ref ** 2))
    linf = float(np.abs(phi - phi_ref).max() / np.abs(phi_ref).max())
    return l1, l2, linf
