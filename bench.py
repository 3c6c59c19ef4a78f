"""Throughput of the HOPE right-hand side on one MI355X.

Workload: 0.25-degree cubed sphere (6 x 360 x 360 cells), genuine 2D WENO of
order 5 (3 Gauss points per edge), FP64, seeded smooth random resting layer
(1000 m + 1 % spherical-harmonic perturbation up to degree 20).  One step is
one SSP-RK3 time step = three right-hand-side evaluations, each a ghost fill,
the panel-edge traces and the fused stage kernel (reconstruction, LMARS,
quadrature, sources, tendency, Runge-Kutta combination).  The state is
resident in HBM before the timed region starts.

Metric: FP64 cell-tendency evaluations per second = interior cells x RHS
evaluations / wall time.  ``value`` is the forward rate; ``fwd_vjp`` holds
the forward+adjoint rates: a tendency plus its vector-Jacobian product on the
same state (one unit per cell), and the 20-step adjoint rollout (forward, then
the backward pass of 0.5 ||h_T - h_target||^2 with checkpoints every 5 steps),
counted as cells x RHS evaluations of the forward over the whole wall time.
Prints one JSON line.
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


def flops_per_cell(order: int, scheme: str, direct: bool = False) -> float:
    """FLOPs of one tendency evaluation of one cell as the fused kernel
    computes it for an owned cell (FMA = 2, add/mul/div/sqrt = 1).

    Per variable: the x-pass at the m+2 axis points (l sub-stencils x (2r+1)
    rows x l taps), the smoothness indicators (an l x l transform per
    sub-stencil and weighted squares), tau and kappa.  The 4m+m^2 point values
    are evaluated by columns: the linear weights factor as gamma = d(py) d(px),
    so per x axis point the sums over sub-stencil columns (l^2 products with
    kappa, l^3 FMAs with the x-pass) are shared by its points, and a point
    costs 2 l^2 + 4 l + 2 where all its gamma are positive and more where the
    split of negative weights is needed (the centre Gauss node of order 5).
    ``direct`` counts the point-by-point evaluation instead (l^2 sub-stencil
    values of l taps each and the split sums per point).  TPP: (2+m) axis
    points x k rows x k taps and k taps per point.  Per cell: LMARS at 2m edge
    points (64 FLOPs + quadrature), sources at m^2 points (43 FLOPs +
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
        if direct:
            points = npts * (2 * s * l + 8 * s + 7)
        else:
            nm = 1 if k == 5 else 0                     # Gauss nodes whose 1D weights change sign
            col = 2 * l * l + 2 * l ** 3
            cols = (2 + m - nm) * col + nm * 2 * col
            n_xm = nm * (2 + m)
            n_ym = 2 * nm + nm * (m - nm)
            n_pos = npts - n_xm - n_ym
            points = cols + n_pos * (2 * l * l + 4 * l + 2) + n_ym * (2 * l * l + 8 * l + 16) \
                + n_xm * (4 * l * l + 8 * l + 16)
        per_var = beta + tau + kappa + xpass + points
    else:
        per_var = (2 + m) * k * 2 * k + npts * 2 * k
    lmars = 2 * m * (64 + 2)
    src = m * m * (43 + 5)
    return 3 * per_var + lmars + src + 15 + 18


# Reference per-cell estimates of the method's arithmetic (separable FMA
# formulation, FMA = 2, add/mul/div/sqrt = 1), independent of this
# implementation's shortcuts: the roofline's headline "achieved" uses these.
REFERENCE_FLOPS_PER_CELL = {("tpp", 3): 1100.0, ("weno", 5): 14800.0, ("tpp", 11): 14100.0}
# the adjoint recomputes the forward point values and applies the transpose
# of every step; its reference estimate is 2.5x the forward (range 2.5-3x)
VJP_FACTOR = 2.5


def reference_flops(order: int, scheme: str):
    return REFERENCE_FLOPS_PER_CELL.get((scheme, order))


STAGE_SOURCES = ("paper_2411_19185_amd/csrc/kernels.hip", "paper_2411_19185_amd/csrc/kernel_bodies.hpp",
                 "paper_2411_19185_amd/csrc/device_common.hpp", "paper_2411_19185_amd/csrc/hope_internal.hpp",
                 "paper_2411_19185_amd/build.py")
TRAFFIC_FILE = "profiles/k_stage_weno5_c360_traffic.txt"


def _cxx_code(src: str) -> str:
    """C++ source text with its comments removed and every run of whitespace
    made one space (string and character literals kept as they are)."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def stage_source_hash() -> str:
    """sha256 over the code of the sources the stage kernel is compiled from
    (comments and layout aside, so that editing a comment keeps the counters
    taken for that code) and the build script with its flags."""
    import hashlib
    h = hashlib.sha256()
    for f in STAGE_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            text = fh.read()
        h.update((text if f.endswith(".py") else _cxx_code(text)).encode())
    return h.hexdigest()[:16]


def measured_traffic(n, order, scheme, launch):
    """HBM bytes per stage launch from the committed counter summary (rocprofv3
    FETCH_SIZE and WRITE_SIZE of the stage kernel, each divided by the factor
    the same counter reads for a copy of known size), or None when the
    summary is missing, is for another workload, or was taken from other
    kernel sources."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    try:
        if kv.get("source_hash") != stage_source_hash():
            return None
        if (int(kv["n"]), int(kv["order"]), kv["scheme"]) != (n, order, scheme):
            return None
        if tuple(int(x) for x in kv["launch"].split(",")) != tuple(launch):
            return None
        return {"bytes_per_launch": float(kv["bytes_per_launch"]), "fetch_bytes": float(kv["fetch_bytes"]),
                "write_bytes": float(kv["write_bytes"]), "copy_factor_fetch": float(kv["copy_factor_fetch"]),
                "copy_factor_write": float(kv["copy_factor_write"])}
    except (KeyError, ValueError):
        return None


COUNTER_FILE = "profiles/hope_weno5_c360_fp64_insts.txt"


def measured_flops(n, order, scheme):
    """Executed FP64 FLOPs per cell of each kernel (lane operations, FMA = 2)
    from the committed counter summary, or None when it is missing, is for
    another workload, or was taken from other kernel sources."""
    path = os.path.join(ROOT, COUNTER_FILE)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    try:
        if kv.get("source_hash") != stage_source_hash():
            return None
        if (int(kv["n"]), int(kv["order"]), kv["scheme"]) != (n, order, scheme):
            return None
        return {k[len("flops_per_cell."):]: float(v) for k, v in kv.items() if k.startswith("flops_per_cell.")}
    except (KeyError, ValueError):
        return None


def cpu_info():
    """Host CPU model, logical CPU count and torch's intra-op thread count."""
    import torch
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "torch_threads": torch.get_num_threads(),
            "torch_version": torch.__version__}


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def copy_calibration():
    """A plain device copy of known size (1 GiB read + 1 GiB written), for
    scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    nbytes = 1 << 30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "copies": 3}), flush=True)


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
    # inside the timed region only the stage kernel carries HIP events (an
    # event between every launch would add a few microseconds each to the step)
    # (the stage's events are recorded by its own launches: no marker between
    # kernels; the timed region holds no other event)
    g.profile(True, only=("stage",))
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    progress(f"C{n} {scheme}{order}: timing {args.steps} SSP-RK3 steps after {args.warmup} warm-up steps")
    evs[0].record(stream)
    for i in range(args.steps):
        g.rk_step(q, dt, "ssp3", ws)
    evs[1].record(stream)
    torch.cuda.synchronize()
    g.profile(False)
    ms = evs[0].elapsed_time(evs[-1])
    # the distribution of single steps, from a second pass with an event after
    # every step (each event costs the stream a few microseconds)
    sev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    sev[0].record(stream)
    for i in range(args.steps):
        g.rk_step(q, dt, "ssp3", ws)
        sev[i + 1].record(stream)
    torch.cuda.synchronize()
    step_ms = sorted(sev[i].elapsed_time(sev[i + 1]) for i in range(args.steps))
    cells = 6 * n * n
    evals = 3 * args.steps
    value = cells * evals / (ms / 1e3)
    st_ms, st_n = g.profile_read("stage")
    traffic = measured_traffic(n, order, scheme, g.get_launch())
    # the ghost fill and panel-edge kernels, timed in a short pass after it
    g.profile(True, only=("fill_halo", "edge_traces"))
    for _ in range(min(args.steps, 5)):
        g.rk_step(q, dt, "ssp3", ws)
    torch.cuda.synchronize()
    g.profile(False)
    halo_ms, halo_n = g.profile_read("fill_halo")
    edge_ms, edge_n = g.profile_read("edge_traces")
    stage_avg = st_ms / max(st_n, 1)
    fpc = flops_per_cell(order, scheme)
    ref_fpc = reference_flops(order, scheme)
    head_fpc = ref_fpc if ref_fpc is not None else fpc
    achieved = head_fpc * cells / (stage_avg / 1e3)
    counters = measured_flops(n, order, scheme)

    def rate(f):
        return {"flops_per_cell": f, "achieved_TFLOPs": f * cells / (stage_avg / 1e3) / 1e12,
                "frac": f * cells / (stage_avg / 1e3) / PEAK_FP64}
    models = {"as_implemented": rate(fpc), "point_by_point": rate(flops_per_cell(order, scheme, direct=True))}
    if counters and "k_stage" in counters:
        models["executed_fp64_counters"] = rate(counters["k_stage"] + counters.get("k_stage_seams", 0.0))
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
        "step_ms": {"median": step_ms[len(step_ms) // 2], "min": step_ms[0], "max": step_ms[-1],
                    "pass": "a second pass of as many steps, an event after every step"},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"C{n} order-{order} {scheme.upper()} SSP-RK3 step, smooth random resting layer",
                   "n": n, "order": order, "scheme": scheme, "cells": cells, "rhs_per_step": 3,
                   "launch": list(g.get_launch()), "dt_s": dt, "seed": args.seed},
        "roofline": {"bound": "alu", "kernel": "k_stage + k_stage_seams (one stage; the events bracket both launches)",
                     "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64,
                     "traffic": None if traffic is None else traffic["bytes_per_launch"],
                     "flops_per_cell": head_fpc,
                     "flop_model": ("reference estimate of the method, separable FMA form (FMA = 2, div/sqrt = 1), "
                                    "x cells per launch" if ref_fpc is not None else "as implemented (bench.flops_per_cell)"),
                     "other_flop_models": models,
                     "traffic_detail": traffic, "stage_source_hash": stage_source_hash(),
                     "stage_avg_ms": stage_avg, "stage_launches": st_n,
                     "hbm_effective_GBps": stage_bytes_per_cell() * cells / (stage_avg / 1e3) / 1e9,
                     "hbm_frac": stage_bytes_per_cell() * cells / (stage_avg / 1e3) / PEAK_HBM},
        "kernels_ms_avg": {"stage": stage_avg, "fill_halo": halo_ms / max(halo_n, 1),
                           "edge_traces": edge_ms / max(edge_n, 1)},
        "state_finite": finite,
        "setup_s": setup_s,
    }
    if not args.no_adjoint:
        progress("forward + adjoint")
        out["fwd_vjp"] = adjoint(g, n, args, dt)
        pair_ms = out["fwd_vjp"]["pair"]["ms"]
        f_pair = head_fpc * (1.0 + VJP_FACTOR)
        ach = f_pair * cells / (pair_ms / 1e3)
        ex = None
        if counters:
            # the tendency's fill, traces and stage, then the adjoint's own fill and kernels
            fill = sum(v for k, v in counters.items() if k.startswith("k_fill_halo"))
            ex = sum(v for k, v in counters.items() if k.startswith("k_vjp") or k in
                     ("k_edge_traces", "k_stage", "k_stage_seams")) + 2 * fill
        out["fwd_vjp"]["roofline"] = {
            "bound": "alu", "kernels": "tendency + hope_tendency_vjp, wall time of the pair",
            "achieved": ach / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s", "frac": ach / PEAK_FP64,
            "flops_per_cell": f_pair,
            "flop_model": f"forward reference estimate x (1 + {VJP_FACTOR}): the adjoint recomputes the "
                          "forward point values and applies the transpose of every step",
            "executed_fp64_flops_per_cell": ex,
            "executed_frac": None if ex is None else ex * cells / (pair_ms / 1e3) / PEAK_FP64}
    if not args.no_tpp11:
        progress("TPP11 C90")
        out["tpp11_c90"] = tpp11(args)
    if not args.no_rh:
        progress("Rossby-Haurwitz wave at C90")
        out["rossby_haurwitz_c90"] = rossby_haurwitz(args)
    if not args.no_ensemble:
        del g
        torch.cuda.empty_cache()
        progress("64-member ensemble")
        out["ensemble"] = ensemble(args)
    if not args.no_cpu_baseline:
        progress("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(qfin, n, order, scheme, args)
    print(json.dumps(out), flush=True)


def tpp11(args):
    """Order-11 TPP at C90 (the differentiation configuration at its timing
    size): forward tendency, its adjoint, and one SSP-RK3 step and its
    adjoint, on the balanced flow with 1e-3 relative noise."""
    import torch

    import hope_inputs as hi
    from paper_2411_19185_amd import Grid, workloads

    n = 90
    f = hi.BalancedFlow(alpha=hi.draw_tilt(args.seed), radius=hi.EARTH_RADIUS)
    q = workloads.cell_average(f, n)
    q = q * (1.0 + 1e-3 * hi.normal_array(args.seed + 1000, q.shape))
    dt = workloads.cfl_dt(q)
    g = Grid(n, 11, "tpp", axis_tilt=f.alpha)
    qp = g.new_state()
    g.interior(qp).copy_(torch.from_numpy(q))
    # the stage's work-item shape, tuned on this grid (order 11 fits one
    # workgroup per CU, so the default shape for order 5 does not carry over)
    from paper_2411_19185_amd import autotune
    autotune.tune_grid(g, qp, cache=args.tune_cache or None)
    w = torch.from_numpy(hi.normal_array(args.seed + 7, (3, 6, n, n))).cuda()
    dq = torch.empty_like(w)
    gq = torch.empty_like(w)
    vws = g.vjp_workspace()
    rws = g.rk_vjp_workspace()
    ws = g.workspace()
    tws = g.tendency_workspace()
    stream = torch.cuda.current_stream()

    def timed(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    t_fwd = timed(lambda: g.tendency(qp, dq, tws))
    t_vjp = timed(lambda: g.tendency_vjp(qp, w, gq, vws))
    qs = qp.clone()
    t_step = timed(lambda: g.rk_step(qs, dt, "ssp3", ws))
    t_step_vjp = timed(lambda: g.rk_step_vjp(qp, dt, w, "ssp3", gq, rws))
    cells = 6 * n * n
    return {"cells": cells, "launch": list(g.get_launch()), "tendency_ms": t_fwd, "tendency_vjp_ms": t_vjp,
            "rk_step_ms": t_step,
            "rk_step_vjp_ms": t_step_vjp, "fwd_value": cells / (t_fwd / 1e3),
            "fwd_vjp_value": cells / ((t_fwd + t_vjp) / 1e3), "unit": "cell-tendency evals/s"}


def ensemble(args):
    """The 64-member uneven ensemble (16 members each at C48, C64, C90, C128,
    WENO5; each a balanced flow with its own axis tilt and a cap jump, its
    own CFL time step): tuned work-item shapes, one captured HIP graph per
    SSP-RK3 step, against looping the single-grid step over the members."""
    import tempfile

    import numpy as np
    import torch

    import hope_inputs as hi
    from paper_2411_19185_amd import Grid, autotune, workloads
    from paper_2411_19185_amd.ensemble import Ensemble

    sizes = (48, 64, 90, 128)
    ns = [sizes[i % 4] for i in range(args.members)]
    t0 = time.time()
    grids = {n: Grid(n, 5, "weno") for n in sizes}
    tilts, states, dts = [], [], []
    for i, n in enumerate(ns):
        f = hi.BalancedFlowWithCap(seed=args.seed * 1000 + i)
        q = workloads.cell_average(f, n)
        tilts.append(f.alpha)
        states.append(q)
        dts.append(workloads.cfl_dt(q))
    ens = Ensemble([grids[n] for n in ns], axis_tilt=tilts)
    q_all = ens.new_state()
    for i, q in enumerate(states):
        ens.member_interior(q_all, i).copy_(torch.from_numpy(q))
    dt = torch.tensor(dts, dtype=torch.float64, device="cuda")
    setup_s = time.time() - t0
    t0 = time.time()
    with tempfile.TemporaryDirectory() as tmp:
        sw, sh, blocks = autotune.tune_ensemble(ens, q_all, cache=args.tune_cache or os.path.join(tmp, "tune.json"))
    tune_s = time.time() - t0
    shapes = {n: [sw[ns.index(n)], sh[ns.index(n)]] for n in sizes}
    cells = sum(6 * n * n for n in ns)
    stream = torch.cuda.current_stream()
    graph = ens.capture_step(q_all, dt)
    for _ in range(2):
        graph.replay()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for _ in range(args.ensemble_steps):
        graph.replay()
    ev[1].record(stream)
    torch.cuda.synchronize()
    batch_ms = ev[0].elapsed_time(ev[1]) / args.ensemble_steps
    finite = bool(torch.isfinite(q_all).all())
    # looped single-grid path (each member's own buffers, the grid of its resolution)
    qps = []
    for i, q in enumerate(states):
        qp = grids[ns[i]].new_state()
        grids[ns[i]].interior(qp).copy_(torch.from_numpy(q))
        qps.append(qp)
    wss = {n: grids[n].workspace() for n in sizes}
    loop_steps = max(1, args.ensemble_steps // 5)
    for i, qp in enumerate(qps):
        grids[ns[i]].rk_step(qp, dts[i], "ssp3", wss[ns[i]])
    torch.cuda.synchronize()
    ev[0].record(stream)
    for _ in range(loop_steps):
        for i, qp in enumerate(qps):
            grids[ns[i]].rk_step(qp, dts[i], "ssp3", wss[ns[i]])
    ev[1].record(stream)
    torch.cuda.synchronize()
    loop_ms = ev[0].elapsed_time(ev[1]) / loop_steps
    # per-member adjoint of the final-state loss 0.5 ||q_T||^2 over the same steps
    vjp_steps = args.ensemble_steps if args.ensemble_vjp else 0
    vjp_ms, grads_finite = 0.0, True
    if vjp_steps:
        q0s = [torch.from_numpy(q).cuda() for q in states]
        for i in range(len(ns)):          # derived member grids, made before timing
            ens.member_grid(i)
        # untimed warm-up (one step): the streams' workspaces are allocated here
        ens.member_loss_gradients(q0s, dts, 1, checkpoint_every=5, streams=args.vjp_streams)
        torch.cuda.synchronize()
        ev[0].record(stream)
        grads = ens.member_loss_gradients(q0s, dts, vjp_steps, checkpoint_every=5, streams=args.vjp_streams)
        ev[1].record(stream)
        grads_finite = all(bool(torch.isfinite(gr).all()) for gr in grads)
        torch.cuda.synchronize()
        vjp_ms = ev[0].elapsed_time(ev[1])
    return {"value": cells * 3 / (batch_ms / 1e3), "unit": "cell-tendency evals/s",
            "members": len(ns), "resolutions": list(sizes), "cells": cells, "steps": args.ensemble_steps,
            "ms_per_step": batch_ms, "state_finite": finite,
            "looped_value": cells * 3 / (loop_ms / 1e3), "looped_ms_per_step": loop_ms, "looped_steps": loop_steps,
            "speedup": loop_ms / batch_ms, "tuned_shapes": shapes, "tuned_blocks": blocks,
            "setup_s": setup_s, "tune_s": tune_s,
            "member_vjp": {"steps": vjp_steps, "checkpoint_every": 5, "ms_total": vjp_ms,
                           "value": (cells * 3 * vjp_steps / (vjp_ms / 1e3)) if vjp_ms else None,
                           "unit": "cell-tendency evals/s (fwd+VJP)", "grads_finite": grads_finite,
                           "loss": "0.5 ||q_T||^2 per member; each member's checkpointed rollout and step "
                                   "adjoints on its own derived grid, members spread over "
                                   f"{args.vjp_streams} HIP streams"},
            "launches_per_step": 12,
            "note": "batched: one captured graph per step (12 kernel launches over all members: ghost fill, "
                    "panel-edge traces, fused stage and segment seams per stage); looped: "
                    "hope_rk_step per member on its resolution's grid (timing only)"}


def rossby_haurwitz(args):
    """The wavenumber-4 Rossby-Haurwitz wave (5.9)-(5.15) at C90 (the grid of
    the paper's order comparison), one SSP-RK3 step per timing, for TPP of
    orders 3, 5 and 7 and WENO5 with their default launch shapes."""
    import torch

    import hope_inputs as hi
    from paper_2411_19185_amd import Grid, workloads

    n = 90
    a = hi.PAPER_RADIUS
    q = workloads.cell_average(hi.RossbyHaurwitz(radius=a), n, radius=a)
    dt = workloads.cfl_dt(q, radius=a)
    cells = 6 * n * n
    stream = torch.cuda.current_stream()
    out = {"cells": cells, "dt_s": dt, "unit": "cell-tendency evals/s", "steps": args.rh_steps, "by_scheme": {}}
    for order, scheme in ((3, "tpp"), (5, "tpp"), (7, "tpp"), (5, "weno")):
        g = Grid(n, order, scheme, radius=a)
        qp = g.new_state()
        g.interior(qp).copy_(torch.from_numpy(q))
        ws = g.workspace()
        for _ in range(3):
            g.rk_step(qp, dt, "ssp3", ws)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        for _ in range(args.rh_steps):
            g.rk_step(qp, dt, "ssp3", ws)
        ev[1].record(stream)
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / args.rh_steps
        out["by_scheme"][f"{scheme}{order}"] = {"ms_per_step": ms, "value": 3 * cells / (ms / 1e3),
                                                "launch": list(g.get_launch()),
                                                "state_finite": bool(torch.isfinite(qp).all())}
        del g, qp, ws
    return out


def adjoint(g, n, args, dt):
    """Forward+adjoint throughput: (1) tendency + hope_tendency_vjp pairs on
    one state, (2) the adjoint rollout of a height-mismatch loss."""
    import numpy as np
    import torch

    import hope_inputs as hi
    from paper_2411_19185_amd import autograd, workloads

    cells = 6 * n * n
    q0 = torch.from_numpy(workloads.smooth_random_state(n, seed=args.seed)).cuda()
    w = torch.from_numpy(hi.normal_array(args.seed + 7, (3, 6, n, n))).cuda()
    qp = g.new_state()
    g.interior(qp).copy_(q0)
    ws = g.vjp_workspace()
    tws = g.tendency_workspace()
    dq = torch.empty(3, 6, n, n, dtype=torch.float64, device="cuda")
    gq = torch.empty_like(dq)
    for _ in range(2):
        g.tendency(qp, dq, tws)
        g.tendency_vjp(qp, w, gq, ws)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    reps = args.vjp_reps
    for _ in range(reps):
        g.tendency(qp, dq, tws)
        g.tendency_vjp(qp, w, gq, ws)
    ev[1].record(stream)
    torch.cuda.synchronize()
    pair_ms = ev[0].elapsed_time(ev[1]) / reps
    # per-kernel times of the adjoint from a second, instrumented pass
    g.profile(True)
    for _ in range(reps):
        g.tendency_vjp(qp, w, gq, ws)
    torch.cuda.synchronize()
    g.profile(False)
    kern = {}
    for k in ("vjp_traces", "vjp_points", "vjp_edges", "vjp_weno", "vjp_gather", "vjp_ghost_t"):
        ms, cnt = g.profile_read(k)
        if cnt:
            kern[k] = ms / reps          # per adjoint call (the WENO adjoint and gather run once per variable)
    fill_ms, fill_cnt = g.profile_read("fill_halo")
    kern["fill_halo"] = fill_ms / max(fill_cnt, 1)
    vjp_ms = sum(v for k, v in kern.items() if k.startswith("vjp_")) + kern["fill_halo"]

    # adjoint rollout
    steps, every = args.rollout_steps, args.checkpoint_every
    sg = torch.from_numpy(workloads.cell_sqrt_g(n)).cuda()
    hscale = 1.0 / (hi.GRAVITY * sg)
    qt = g.new_state()
    g.interior(qt).copy_(torch.from_numpy(workloads.smooth_random_state(n, seed=args.seed + 1)))
    rws = g.workspace()
    for _ in range(steps):
        g.rk_step(qt, dt, "ssp3", rws)
    h_target = (g.interior(qt)[0] * hscale).contiguous()
    del qt, rws, qp, ws, dq, gq
    # untimed warm-up: one checkpoint segment forward and backward, so that the
    # timed run does not include the first device allocation of its workspaces
    qw = q0.clone().requires_grad_(True)
    (0.5 * (autograd.rollout(g, qw, dt, min(steps, every), checkpoint_every=every) ** 2).sum()).backward()
    del qw
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    base_mem = torch.cuda.memory_allocated()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    q = q0.clone().requires_grad_(True)
    ev[0].record(stream)
    qT = autograd.rollout(g, q, dt, steps, checkpoint_every=every)
    ev[1].record(stream)
    loss = 0.5 * ((qT[0] * hscale - h_target) ** 2).sum()
    loss.backward()
    ev[2].record(stream)
    torch.cuda.synchronize()
    fwd_ms = ev[0].elapsed_time(ev[1])
    bwd_ms = ev[1].elapsed_time(ev[2])
    peak = torch.cuda.max_memory_allocated() - base_mem
    grad_finite = bool(torch.isfinite(q.grad).all())
    return {
        "pair": {"value": cells / (pair_ms / 1e3), "unit": "cell-(tendency+VJP) evals/s", "ms": pair_ms,
                 "vjp_ms": vjp_ms, "kernels_ms_avg": kern, "reps": reps},
        "rollout": {"value": cells * 3 * steps / ((fwd_ms + bwd_ms) / 1e3), "unit": "cell-tendency evals/s (fwd+VJP)",
                    "steps": steps, "checkpoint_every": every, "fwd_ms": fwd_ms, "bwd_ms": bwd_ms,
                    "fwd_value": cells * 3 * steps / (fwd_ms / 1e3),
                    "peak_device_bytes_torch": int(peak), "grid_device_bytes": int(g.layout.device_bytes),
                    "loss": float(loss), "grad_finite": grad_finite,
                    "target": f"forward state after {steps} steps from seed {args.seed + 1}"},
    }


def cpu_baseline(q, n, order, scheme, args, evals=2):
    """The FP64 oracle on the host cores, as it stands (not tuned): full
    right-hand-side evaluations (ghost fixed point, reconstruction, LMARS,
    quadrature) of the benchmark grid and its final state on all threads
    (the headline value); one evaluation at C90 of the same scheme on one
    thread; and the oracle's autograd adjoint (forward + backward of
    <w, dq/dt>) at C12 and C90 TPP11 and at C90 WENO5."""
    import torch

    import hope_inputs as hi
    from oracle.ic import cell_average
    from oracle.rhs import Grid as OracleGrid
    from oracle.rhs import Params
    info = cpu_info()
    threads = torch.get_num_threads()
    og = OracleGrid(n, order, scheme, Params())
    t0 = time.time()
    for _ in range(evals):
        og.tendency(q)
    sec = time.time() - t0
    out = {"value": evals * 6 * n * n / sec, "unit": "cell-tendency evals/s", "cores": threads, "kind": "oracle",
           "sample": f"{evals} full RHS evaluations at C{n} (6x{n}x{n} cells) of the final benchmark state, "
                     f"{sec:.1f} s on {threads} threads", **info}
    if args.cpu_extra:
        radius = hi.EARTH_RADIUS
        q90 = cell_average(hi.RestingLayer(seed=args.seed, with_cap=False), 90, radius, nq=2)
        og90 = OracleGrid(90, order, scheme, Params())
        torch.set_num_threads(1)
        try:
            t0 = time.time()
            og90.tendency(q90)
            sec1 = time.time() - t0
        finally:
            torch.set_num_threads(threads)
        out["one_thread"] = {"value": 6 * 90 * 90 / sec1, "unit": "cell-tendency evals/s", "cores": 1,
                             "sample": f"1 RHS evaluation at C90 {scheme.upper()}{order}, {sec1:.1f} s"}
        vjp = {}
        for nn, k, sch in ((12, 11, "tpp"), (90, 11, "tpp"), (90, 5, "weno")):
            f = hi.BalancedFlow(alpha=hi.draw_tilt(args.seed), radius=radius)
            qq = cell_average(f, nn, radius, nq=2)
            qq = qq * (1.0 + 1e-3 * torch.tensor(hi.normal_array(args.seed + 1000, tuple(qq.shape))))
            w = torch.tensor(hi.normal_array(args.seed + 7, tuple(qq.shape)))
            ogv = OracleGrid(nn, k, sch, Params(alpha=f.alpha))
            x = qq.clone().requires_grad_(True)
            t0 = time.time()
            (ogv.tendency(x) * w).sum().backward()
            secv = time.time() - t0
            vjp[f"C{nn}_{sch}{k}"] = {"value": 6 * nn * nn / secv, "unit": "cell-(tendency+VJP) evals/s",
                                      "seconds": secv, "cores": threads}
        out["autograd_vjp"] = vjp
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=360)
    ap.add_argument("--order", type=int, default=5)
    ap.add_argument("--scheme", default="weno")
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--launch", default="", help="strip_w,seg_h of the stage kernel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-tpp11", action="store_true")
    ap.add_argument("--no-rh", action="store_true", help="skip the Rossby-Haurwitz throughput section")
    ap.add_argument("--rh-steps", type=int, default=20)
    ap.add_argument("--no-cpu-extra", dest="cpu_extra", action="store_false",
                    help="CPU baseline: only the headline all-thread forward evaluations")
    ap.add_argument("--tune-cache", default="", help="autotuner cache file (default: a fresh one per run)")
    ap.add_argument("--members", type=int, default=64)
    ap.add_argument("--ensemble-steps", type=int, default=50)
    ap.add_argument("--no-ensemble-vjp", dest="ensemble_vjp", action="store_false")
    ap.add_argument("--vjp-streams", type=int, default=8, help="HIP streams for the per-member adjoints")
    ap.add_argument("--copy-calibration", action="store_true", help="only run a 1 GiB device copy (counter scale)")
    ap.add_argument("--vjp-reps", type=int, default=10)
    ap.add_argument("--rollout-steps", type=int, default=20)
    ap.add_argument("--checkpoint-every", type=int, default=5)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU panel "
              "decomposition is a design, not built", file=sys.stderr)
        raise SystemExit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    run(args)


if __name__ == "__main__":
    main()
