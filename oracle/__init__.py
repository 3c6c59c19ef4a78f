"""Plain FP64 CPU oracle for the HOPE right-hand side (arXiv 2411.19185).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the tests, the smoke check and the CPU-baseline leg of the benchmark use it.

It is written from the paper, step by step, in double precision with
PyTorch CPU tensors (so that ``torch.autograd`` over it is an independent
reference gradient), with exact rational / multiprecision construction of the
reconstruction weights.  It shares no code with the GPU path.

Modules
  weights   1D/2D cell-average -> point weights (3.7)-(3.15), Gauss rules
            (3.5)-(3.6), WENO linear weights (3.16)-(3.20), smoothness
            indicator forms (3.25)
  geometry  panel maps, metric (2.5)-(2.8), wind conversion J (2.10)-(2.12)
  ghost     iterative ghost-cell interpolation, section 3.3.1 and (7.1)-(7.12)
  rhs       reconstruction, panel-boundary conversion (3.26)-(3.29), LMARS
            (3.30)-(3.38), quadrature and sources, tendency (3.1)
  rk        three-stage Runge-Kutta (section 3.5)
  ic        projection of the shared physical test fields onto cell averages
  norms     mass and the error norms (5.4)-(5.7)

Every reading of a garbled or silent passage is listed in ``READINGS``.
"""

READINGS = {
    "metric_denominator": "(2.6) denominator read as (1+X^2)(1+Y^2): the only inverse of (2.7)",
    "flux_difference": "(3.1) read as F(i+1/2)-F(i-1/2); Delta = pi/(2N) angular spacing",
    "gauss_points": "m = (k+1)/2 Gauss points per edge, m*m per cell, weights sum to 1",
    "split_combination": "(3.21) read as sigma+ sum w+ p - sigma- sum w- p, sigma = sum gamma",
    "split_everywhere": "the negative-weight split is applied at every point",
    "weno_epsilon": "WENO epsilon = 1e-12 applied to beta of the stored variables",
    "weno_z_tau": "(3.24) tau = 2/(s(s+1)) * sum over pairs eta<psi |beta_psi-beta_eta|",
    "smoothness_indicator": "(3.25) beta = sum over derivative orders (a,b)!=(0,0), a,b<=l-1, "
           "of the integral over the unit target cell of the squared derivative",
    "weno_at_cqp": "the same WENO is applied at the cell quadrature points",
    "weno_variables": "WENO acts component-wise on (sqrtG phi, sqrtG phi u, sqrtG phi v)",
    "ghost_linear": "ghost cells always use the linear order-k TPP, also in WENO mode",
    "ghost_owner": "ghost GQP owner panel = largest signed Cartesian component; on an "
           "exact tie (diagonal of a corner ghost block) the two owners' "
           "converted interpolants are averaged; containing cell by floor, "
           "clamped; central k x k stencil in the owner's padded array",
    "ghost_fixed_point": "ghost fixed point iterated until the relative change of every "
           "variable is below 1e-15, then three more sweeps",
    "ghost_conversion_order": "interpolate in the owner's variables, convert at each GQP, then average",
    "panel_edge_flux": "at a panel-edge EQP the outside state is the neighbour panel's own "
           "inner trace, converted; each panel evaluates its own flux",
    "lmars_upwind": "(3.37) upwind term read as |m| (q_R - q_L)",
    "lmars_pressure": "pressure term of (3.38) uses phi* of (3.33)",
    "time_scheme": "SSP-RK3 (Shu-Osher) by default; the printed Wicker-Skamarock scheme "
           "with (3.40) read as q** = q^n + dt/2 L(q*)",
    "tilted_coriolis": "Coriolis parameter f = 2 Omega (Omega_hat . p) with the axis tilted "
           "by alpha, Omega_hat = (-sin alpha, 0, cos alpha)",
    "norms_abs": "norms (5.4)-(5.7) with absolute values",
}
