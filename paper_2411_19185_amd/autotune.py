"""Autotuner of the fused stage kernel's work-item shape (strip width and
segment height) and, for ensembles, of the stage launch's grid size.

Every candidate gives bitwise identical results, so tuning is a pure timing
search: each candidate is timed with HIP events around the library's own
calls on the current stream (median of a few repetitions), and the fastest
is kept.  Results are cached in a JSON file keyed by the device, order,
scheme and resolution(s), so a tuned shape is reused by later processes.

Cache file: the ``cache`` argument, else $HOPE_AUTOTUNE_CACHE, else
~/.cache/hope/autotune.json.
"""
from __future__ import annotations

import json
import os
import statistics

import torch

SEG_CANDIDATES = (2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 14, 16, 20, 24, 32)


def _cache_path(cache: str | None) -> str:
    return cache or os.environ.get("HOPE_AUTOTUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "hope", "autotune.json")


def _load(path: str) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path: str, data: dict):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


HALF_STRIP = 30   # strips this narrow run two per workgroup (32 lanes each)


def strip_candidates(n: int) -> list[int]:
    """Strip widths, each balanced over the panel: those <= 62 that split n
    into 1..4 more strips than needed, and those <= 30 (two strips per
    workgroup) that split it into 1..3 more than needed at that width."""
    out = []
    for cap, extra in ((62, 4), (HALF_STRIP, 3)):
        need = (n + cap - 1) // cap
        for strips in range(need, need + extra):
            w = (n + strips - 1) // strips
            if 1 <= w <= 62 and w not in out:
                out.append(w)
    return out


def _time(fn, reps: int) -> float:
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return statistics.median(ts)


def _device_key() -> str:
    # the architecture name (the marketing name can read empty under a profiler)
    props = torch.cuda.get_device_properties(0)
    name = getattr(props, "gcnArchName", "") or torch.cuda.get_device_name(0) or "gpu"
    return name.split(":")[0].replace("|", "/")


def tune_grid(grid, q: torch.Tensor, reps: int = 5, cache: str | None = None, force: bool = False):
    """Best (strip_w, seg_h) for one grid, timed on hope_tendency of the
    padded state q; applied to the grid and returned."""
    path = _cache_path(cache)
    key = f"grid|{_device_key()}|{grid.order}|{grid.scheme}|{grid.n}"
    data = _load(path)
    if key in data and not force:
        sw, sh = data[key]["launch"]
        grid.set_launch(sw, sh)
        return sw, sh
    out = torch.empty(3, 6, grid.n, grid.n, dtype=torch.float64, device="cuda")
    best = None
    for sw in strip_candidates(grid.n):
        for sh in SEG_CANDIDATES:
            if sh > grid.n:
                continue
            grid.set_launch(sw, sh)
            ws = grid.tendency_workspace()             # its size depends on the segment height
            grid.tendency(q, out, ws)                  # warm
            t = _time(lambda: grid.tendency(q, out, ws), reps)
            if best is None or t < best[0]:
                best = (t, sw, sh)
    _, sw, sh = best
    grid.set_launch(sw, sh)
    data = _load(path)
    data[key] = {"launch": [sw, sh], "ms": best[0]}
    _store(path, data)
    return sw, sh


def tune_ensemble(ens, q_all: torch.Tensor, reps: int = 5, cache: str | None = None, force: bool = False,
                  blocks_candidates=(0, 1024, 2048, 4096), passes: int = 2):
    """Per-resolution (strip_w, seg_h) and the stage grid size for an
    ensemble, timed on the batched tendency of q_all: coordinate descent over
    the resolutions (all members of one grid share a shape; ``passes`` rounds,
    each resolution searched again with the others at their latest shapes),
    then over the grid size.  Applied to the ensemble and returned as
    (strip_w, seg_h, blocks) lists per member."""
    path = _cache_path(cache)
    ns = [g.n for g in ens.grids]
    groups: dict[int, list[int]] = {}
    for i, g in enumerate(ens.grids):
        groups.setdefault(id(g), []).append(i)
    sig = sorted((ens.grids[m[0]].n, len(m)) for m in groups.values())
    g0 = ens.grids[0]
    key = f"batch|{_device_key()}|{g0.order}|{g0.scheme}|{sig}"
    data = _load(path)
    if key in data and not force:
        per_n = {int(k): v for k, v in data[key]["shapes"].items()}
        sw = [per_n[n][0] for n in ns]
        sh = [per_n[n][1] for n in ns]
        ens.set_launch(sw, sh, data[key]["blocks"])
        return sw, sh, data[key]["blocks"]
    out = ens.new_field()
    sw, sh, blocks = ens.get_launch()

    def run():
        ens.tendency(q_all, out)

    for _ in range(max(1, passes)):
        for members in groups.values():
            n = ens.grids[members[0]].n
            best = None
            for cw in strip_candidates(n):
                for ch in SEG_CANDIDATES:
                    if ch > n:
                        continue
                    for i in members:
                        sw[i], sh[i] = cw, ch
                    ens.set_launch(sw, sh, blocks)
                    run()
                    t = _time(run, reps)
                    if best is None or t < best[0]:
                        best = (t, cw, ch)
            for i in members:
                sw[i], sh[i] = best[1], best[2]
    best = None
    for b in blocks_candidates:
        ens.set_launch(sw, sh, b)
        run()
        t = _time(run, reps)
        if best is None or t < best[0]:
            best = (t, b)
    blocks = best[1]
    ens.set_launch(sw, sh, blocks)
    shapes = {}
    for i, n in enumerate(ns):
        shapes[str(n)] = [sw[i], sh[i]]
    data = _load(path)
    data[key] = {"shapes": shapes, "blocks": blocks, "ms": best[0]}
    _store(path, data)
    return sw, sh, blocks
