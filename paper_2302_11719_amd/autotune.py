"""Launch-geometry autotuner for the batched plan.

The fused kernel of a plan has four knobs: the four-wave latency mode
(``pipeline``), the workgroup size (``block``: 64, 128, 256, 512), the samples
per tile (``tile`` = block x samples-per-thread, 1, 2 or 4) and the number of
persistent workgroups (``grid``; 0 = the occupancy limit).  Which is fastest
depends on the batch shape: a few thousand samples are bound by the per-step
dependency chain of each wave (latency mode wins), hundreds of thousands by
VALU issue (large blocks, one sample per lane), ragged batches by the tail of
the tile queue.

``tune`` times every candidate on the caller's batch with kernel-stamped events
(the fused kernel alone, eager launches of the plan) and keeps the fastest;
results are cached in a JSON file keyed by the batch shape and the device's
compute-unit count, so a later ``tuned_plan`` for the same shape costs one
file read.  Plans built here own their outputs; tuning never writes the
caller's state, controls or counters.
"""
from __future__ import annotations

import json
import math
import os
import tempfile
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
import torch

from . import core

DEFAULT_CACHE = os.environ.get("SMPPI_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "smppi", "autotune.json"))
BLOCKS = (64, 128, 256, 512)
SPTS = (1, 2, 4)
GRID_MULTS = (0, 1, 2, 4)  # 0: occupancy-derived; otherwise that many workgroups per CU


@dataclass
class TuneResult:
    key: str
    best: Dict[str, int]
    best_ms: float
    table: List[dict] = field(default_factory=list)
    cached: bool = False


def _n_cu(ctx: core.Context) -> int:
    return torch.cuda.get_device_properties(ctx.device).multi_processor_count


def shape_key(db: core.DeviceBatch, n_cu: int) -> str:
    """Batch shape signature: B, total samples (to 1/8 octave), largest K and T,
    mean T, obstacles present, compute units."""
    K = np.asarray(db.K, dtype=np.int64)
    T = np.asarray(db.T, dtype=np.int64)
    sum_k = int(K.sum())
    octave = round(8 * math.log2(sum_k)) if sum_k > 0 else -1
    obs = int(db.track.obs_max > 0)
    return (f"B{db.B}-sk{octave}-kmax{int(K.max(initial=0))}-tmax{int(T.max(initial=0))}"
            f"-tmean{float(T.mean()) if len(T) else 0:.1f}-obs{obs}-cu{n_cu}")


def candidates(n_cu: int) -> List[Dict[str, int]]:
    out = [dict(pipeline=1, block=0, tile=0, grid=0)]
    for block in BLOCKS:
        for spt in SPTS:
            if block * spt > 1024:
                continue
            for gm in GRID_MULTS:
                out.append(dict(pipeline=-1, block=block, tile=block * spt, grid=gm * n_cu))
    return out


def _time_candidate(ctx, db, model, cost, seed, lam, cand, reps, warmup) -> float:
    plan = core.Plan(ctx, db, model, cost, seed, lam, use_graph=False, **cand)
    try:
        ms = []
        for i in range(warmup + reps):
            plan.launch_profiled()
            f, _ = plan.kernel_ms()
            if i >= warmup:
                ms.append(f)
        return float(np.median(ms))
    finally:
        plan.close()


def _load(path: Optional[str]) -> dict:
    if not path or not os.path.exists(path):
        return {}
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path: str, data: dict) -> None:
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".autotune-")
    with os.fdopen(fd, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(ctx: core.Context, db: core.DeviceBatch, model: dict, cost: dict, seed: int, lam: float, *,
         cands: Optional[List[Dict[str, int]]] = None, reps: int = 5, warmup: int = 2,
         cache: Optional[str] = DEFAULT_CACHE, force: bool = False) -> TuneResult:
    """Time each candidate geometry on this batch; return the fastest (and the table).

    With a cache path, a stored result for the same shape key is returned without
    timing unless ``force``; a new result is merged into the file."""
    n_cu = _n_cu(ctx)
    key = shape_key(db, n_cu)
    store = _load(cache)
    if not force and key in store:
        e = store[key]
        return TuneResult(key, e["best"], e["best_ms"], e.get("table", []), cached=True)
    steps = int(sum(k * t for k, t in zip(db.K, db.T)))
    table = []
    for cand in (cands if cands is not None else candidates(n_cu)):
        ms = _time_candidate(ctx, db, model, cost, seed, lam, cand, reps, warmup)
        table.append(dict(cand, kernel_ms=ms, rollout_steps_per_s=steps / (ms * 1e-3) if ms > 0 else None))
    table.sort(key=lambda r: r["kernel_ms"])
    best = {k: table[0][k] for k in ("pipeline", "block", "tile", "grid")}
    res = TuneResult(key, best, table[0]["kernel_ms"], table)
    if cache:
        store = _load(cache)
        store[key] = {"best": best, "best_ms": res.best_ms, "table": table}
        _store(cache, store)
    return res


def tuned_plan(ctx: core.Context, db: core.DeviceBatch, model: dict, cost: dict, seed: int, lam: float, *,
               cache: Optional[str] = DEFAULT_CACHE, **plan_kwargs) -> core.Plan:
    """A plan with the tuned geometry for this batch shape (tuning first if the
    cache has no entry).  ``plan_kwargs`` are the other Plan options (repair,
    execute, dist, use_graph, nominal)."""
    res = tune(ctx, db, model, cost, seed, lam, cache=cache)
    return core.Plan(ctx, db, model, cost, seed, lam, **res.best, **plan_kwargs)
