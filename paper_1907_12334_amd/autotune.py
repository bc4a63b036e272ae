"""Plan autotuner: picks the smoother tile shape and the on-chip tail depth
budget for a workload by timing the library on a slice of it.

The plan parameters (msg_solve_opts.tail_budget, tile_width, tile_cells,
tile_lds) change neither the arithmetic nor the results beyond rounding; they
trade LDS per workgroup against halo traffic and resident problems per CU,
which is a property of the batch size and grid shapes rather than something
the library can derive.  Each trial runs a bounded number of cycles
(max_cycles) of the full-MSG solve on `samples` samples of the workload with
fields already on the device, timed from the host around the call; the
search is coordinate-wise (tile shape first, then the tail budget), keeping
the fastest.  Results can be cached in a JSON file keyed by the workload's
shape.  Nothing here computes any part of the method.
"""
from __future__ import annotations

import dataclasses
import json
import os
import time
from typing import Dict, List, Optional, Sequence, Tuple

from . import inputs as I
from . import msg

# (tile_width, tile_cells, tile_lds): the library default first
TILES: Tuple[Tuple[int, int, int], ...] = ((64, 1024, 2048), (32, 512, 2048), (64, 512, 2048), (128, 1024, 4096),
                                           (64, 2048, 4096))
TAIL_BUDGETS: Tuple[int, ...] = (20480, 12288, 28672, 40960)


# wider tail budgets, for batches of few problems per class (ragged batches,
# the request loop), where each level kept on chip saves host level visits
WIDE_TAIL_BUDGETS: Tuple[int, ...] = (20480, 40960, 65536, 102400, 153600)


def shape_key(w: I.Workload, samples: int, precision: int) -> str:
    return (f"c{w.c}-P{min(w.P)}..{max(w.P)}-Q{min(w.Q)}..{max(w.Q)}-S{samples}-"
            f"{'mixed' if precision == msg.MIXED else 'fp64'}")


def _trial(h, w: I.Workload, opts: msg.SolveOpts, xi, reps: int) -> float:
    import torch
    batch = msg.Batch(w.c, w.P, w.Q)
    bufs = msg.Buffers(batch, opts)
    h.sample_field(msg.FieldSpec(w.field), batch, xi, bufs.kx, bufs.ky, bufs.kx32, bufs.ky32)
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.solve_batch(batch, opts, bufs.kx, bufs.ky, bufs.kx32, bufs.ky32, None, bufs.u, bufs.q, bufs.status,
                      bufs.cycles, bufs.ws)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    del bufs
    return best


def autotune(h: msg.Handle, w: I.Workload, opts: msg.SolveOpts, samples: int = 1024, cycles: int = 2,
             reps: int = 2, cache: Optional[str] = None, log=None, margin: float = 0.02,
             budgets: Sequence[int] = TAIL_BUDGETS, overlaps: Sequence[int] = ()) -> Tuple[msg.SolveOpts, dict]:
    """Returns (opts with the fastest plan parameters, report).  A candidate
    replaces the current choice only when it is faster by more than `margin`
    (relative), so timing noise does not move the plan off the defaults.
    `budgets` are the tail budgets tried (the first is the starting point);
    `overlaps`, if given, the overlap modes tried last (results do not depend
    on them either)."""
    import torch
    sub = w.subset(min(samples, w.n_samples))
    key = shape_key(w, sub.n_samples, opts.precision)
    if cache and os.path.exists(cache):
        try:
            hit = json.load(open(cache)).get(key)
        except (OSError, ValueError):
            hit = None
        if hit:
            return dataclasses.replace(opts, **hit["params"]), dict(hit, cached=True)
    xi = torch.tensor(sub.xi(), dtype=torch.float64, device=f"cuda:{h.device}")
    trial_opts = dataclasses.replace(opts, max_cycles=cycles)
    trials: List[dict] = []

    def run(params: Dict[str, int]) -> float:
        t = _trial(h, sub, dataclasses.replace(trial_opts, **params), xi, reps)
        trials.append({"params": dict(params), "seconds": round(t, 4)})
        if log:
            log(f"autotune {params}: {t:.3f} s")
        return t

    best_params = {"tail_budget": budgets[0], "tile_width": TILES[0][0], "tile_cells": TILES[0][1],
                   "tile_lds": TILES[0][2]}
    best = run(best_params)
    for tw, cells, lds in TILES[1:]:
        p = dict(best_params, tile_width=tw, tile_cells=cells, tile_lds=lds)
        t = run(p)
        if t < best * (1.0 - margin):
            best, best_params = t, p
    for tb in budgets[1:]:
        p = dict(best_params, tail_budget=tb)
        t = run(p)
        if t < best * (1.0 - margin):
            best, best_params = t, p
    if overlaps:
        best_params = dict(best_params, overlap=overlaps[0])
        best = run(best_params)
        for ov in overlaps[1:]:
            p = dict(best_params, overlap=ov)
            t = run(p)
            if t < best * (1.0 - margin):
                best, best_params = t, p
    report = {"key": key, "params": best_params, "seconds": round(best, 4), "samples": sub.n_samples,
              "cycles_per_trial": cycles, "margin": margin, "trials": trials, "cached": False}
    if cache:
        try:
            data = json.load(open(cache)) if os.path.exists(cache) else {}
        except (OSError, ValueError):
            data = {}
        data[key] = {k: report[k] for k in ("key", "params", "seconds", "samples", "cycles_per_trial")}
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(data, f, indent=1)
    return dataclasses.replace(opts, **best_params), report
