"""Pins of the oracle's gradient (torch autograd over the FP64 oracle, the
reference the hand-written adjoint is compared with): the directional
derivative <dL/dq, v> against a central finite difference of the oracle
itself, for the tendency and for one SSP-RK3 step, with the relative step
of each component that the differentiation experiment uses."""
import pytest
import torch

import hope_inputs as hi
from cases import STATES, cfl_dt, oracle_grid
from oracle.rk import ssp_rk3


@pytest.mark.parametrize("n,order,scheme,state,seed", [(6, 3, "tpp", "member", 60), (6, 3, "weno", "member", 61),
                                                       (6, 5, "weno", "perturbed_balanced", 62),
                                                       (7, 7, "tpp", "perturbed_balanced", 63)])
def test_oracle_autograd_matches_central_difference(n, order, scheme, state, seed):
    alpha, q = STATES[state](n, seed)
    og = oracle_grid(n, order, scheme, alpha)
    w = torch.tensor(hi.normal_array(seed + 1, tuple(q.shape)))
    v = q * torch.tensor(hi.normal_array(seed + 2, tuple(q.shape)))
    qq = q.clone().requires_grad_(True)
    (og.tendency(qq) * w).sum().backward()
    ad = float((qq.grad * v).sum())
    h = 1e-6
    fd = float(((og.tendency(q + h * v) - og.tendency(q - h * v)) * w).sum() / (2 * h))
    assert abs(ad - fd) <= 1e-7 * abs(ad), (ad, fd)


def test_oracle_rk_step_autograd_matches_central_difference():
    n, order, scheme = 6, 5, "tpp"
    alpha, q = STATES["member"](n, 64)
    og = oracle_grid(n, order, scheme, alpha)
    dt = cfl_dt(q)
    w = torch.tensor(hi.normal_array(65, tuple(q.shape)))
    v = q * torch.tensor(hi.normal_array(66, tuple(q.shape)))
    qq = q.clone().requires_grad_(True)
    (ssp_rk3(og.tendency, qq, dt) * w).sum().backward()
    ad = float((qq.grad * v).sum())
    h = 1e-6
    fd = float(((ssp_rk3(og.tendency, q + h * v, dt) - ssp_rk3(og.tendency, q - h * v, dt)) * w).sum() / (2 * h))
    assert abs(ad - fd) <= 1e-7 * abs(ad), (ad, fd)
