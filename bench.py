"""Throughput of the HOPE right-hand side on one MI355X.

Workload: 0.25-degree cubed sphere (6 x 360 x 360 cells), genuine 2D WENO of
order 5 (3 Gauss points per edge), FP64, seeded smooth random resting layer
(1000 m + 1 % spherical-harmonic perturbation up to degree 20).  One step is
one SSP-RK3 time step = three right-hand-side evaluations, each a ghost fill,
the panel-edge traces and the fused stage kernel (reconstruction, LMARS,
quadrature, sources, tendency, Runge-Kutta combination).  The state is
resident in HBM before the timed region starts.

Metric: FP64 cell-tendency evaluations per second = interior cells x RHS
evaluations / wall time.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12        # MI355X FP64 vector, FLOP/s
PEAK_HBM = 8.0e12          # bytes/s


def flops_per_cell(order: int, scheme: str) -> float:
    """FLOPs of one tendency evaluation of one cell as the fused kernel
    computes it for an owned cell (FMA = 2, add/mul/div/sqrt = 1).

    Per variable: WENO x-pass 5 axis points x l sub-stencils x (2r+1) rows x l
    taps, and for every one of the 4m+m^2 points l^2 sub-stencil values (l
    taps) plus the split combination; smoothness indicators by an l x l
    transform per sub-stencil and weighted squares; tau and kappa.  TPP: (2+m)
    axis points x k rows x k taps and k taps per point.  Per cell: LMARS at 2m
    edge points (64 FLOPs + quadrature), sources at m^2 points (43 FLOPs +
    quadrature), assembly and the Runge-Kutta combination.
    """
    k = order
    m = (k + 1) // 2
    r = (k - 1) // 2
    npts = 4 * m + m * m
    if scheme == "weno":
        l = (k + 1) // 2
        s = l * l
        beta = 2 * (l * (2 * r + 1) * l * l) + 2 * (s * (s - 1) * l) + 3 * s * (s - 1)
        tau = 2 * (s * (s - 1) // 2) + 1
        kappa = 3 * s
        xpass = (2 + m) * l * (2 * r + 1) * 2 * l
        point = 2 * s * l + 8 * s + 7
        per_var = beta + tau + kappa + xpass + npts * point
    else:
        per_var = (2 + m) * k * 2 * k + npts * 2 * k
    lmars = 2 * m * (64 + 2)
    src = m * m * (43 + 5)
    return 3 * per_var + lmars + src + 15 + 18


def stage_bytes_per_cell() -> float:
    """Algorithmic HBM bytes of one fused stage per cell: read q_s and q_n,
    write q_{s+1} (3 FP64 each)."""
    return 72.0


def run(args):
    import numpy as np
    import torch

    from paper_2411_19185_amd import Grid, workloads

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU (the HIP library has no CPU path)")
    n, order, scheme = args.n, args.order, args.scheme
    t0 = time.time()
    q0 = workloads.smooth_random_state(n, seed=args.seed)
    dt = workloads.cfl_dt(q0)
    g = Grid(n, order, scheme)
    if args.launch:
        sw, sh = (int(v) for v in args.launch.split(","))
        g.set_launch(sw, sh)
    setup_s = time.time() - t0
    q = g.new_state()
    g.interior(q).copy_(torch.from_numpy(q0))
    ws = g.workspace()
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        g.rk_step(q, dt, "ssp3", ws)
    torch.cuda.synchronize()
    g.profile(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        g.rk_step(q, dt, "ssp3", ws)
    ev1.record(stream)
    torch.cuda.synchronize()
    g.profile(False)
    ms = ev0.elapsed_time(ev1)
    cells = 6 * n * n
    evals = 3 * args.steps
    value = cells * evals / (ms / 1e3)
    st_ms, st_n = g.profile_read("stage")
    halo_ms, halo_n = g.profile_read("fill_halo")
    edge_ms, edge_n = g.profile_read("edge_traces")
    stage_avg = st_ms / max(st_n, 1)
    fpc = flops_per_cell(order, scheme)
    achieved = fpc * cells / (stage_avg / 1e3)
    qfin = g.interior(q).double().cpu()
    finite = bool(torch.isfinite(qfin).all())
    out = {
        "metric": "FP64 cell-tendency evals/s (fwd) at 0.25 deg WENO5",
        "value": value,
        "unit": "cell-tendency evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"C{n} order-{order} {scheme.upper()} SSP-RK3 step, smooth random resting layer",
                   "n": n, "order": order, "scheme": scheme, "cells": cells, "rhs_per_step": 3,
                   "launch": list(g.get_launch()), "dt_s": dt, "seed": args.seed},
        "roofline": {"bound": "alu", "kernel": "k_stage", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": None,
                     "flops_per_cell": fpc, "stage_avg_ms": stage_avg, "stage_launches": st_n,
                     "hbm_effective_GBps": stage_bytes_per_cell() * cells / (stage_avg / 1e3) / 1e9,
                     "hbm_frac": stage_bytes_per_cell() * cells / (stage_avg / 1e3) / PEAK_HBM},
        "kernels_ms_avg": {"stage": stage_avg, "fill_halo": halo_ms / max(halo_n, 1),
                           "edge_traces": edge_ms / max(edge_n, 1)},
        "state_finite": finite,
        "setup_s": setup_s,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(qfin, n, order, scheme)
    print(json.dumps(out), flush=True)


def cpu_baseline(q, n, order, scheme):
    """The FP64 oracle on the host cores: one full right-hand-side evaluation
    (ghost fixed point, reconstruction, LMARS, quadrature) of the same grid
    and state."""
    import torch

    from oracle.rhs import Grid as OracleGrid
    from oracle.rhs import Params
    threads = torch.get_num_threads()
    og = OracleGrid(n, order, scheme, Params())
    t0 = time.time()
    og.tendency(q)
    sec = time.time() - t0
    return {"value": 6 * n * n / sec, "unit": "cell-tendency evals/s", "cores": threads, "kind": "oracle",
            "sample": f"one full RHS evaluation at C{n} (6x{n}x{n} cells), {sec:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=360)
    ap.add_argument("--order", type=int, default=5)
    ap.add_argument("--scheme", default="weno")
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--launch", default="", help="strip_w,seg_h of the stage kernel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU panel "
              "decomposition is a design, not built", file=sys.stderr)
        raise SystemExit(2)
    run(args)


if __name__ == "__main__":
    main()
