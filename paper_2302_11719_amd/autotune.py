"""Launch-geometry autotuner for the batched plan.

The fused kernel of a plan has four knobs: the four-wave latency mode
(``pipeline``), the workgroup size (``block``: 64, 128, 256, 512), the samples
per tile (``tile`` = block x samples-per-thread, 1, 2 or 4) and the number of
persistent workgroups (``grid``; 0 = the occupancy limit).  Which is fastest
depends on the batch shape: a few thousand samples are bound by the per-step
dependency chain of each wave (latency mode wins), hundreds of thousands by
VALU issue (large blocks, one sample per lane), ragged batches by the tail of
the tile queue.

``tune`` calls ``smppi_autotune`` of the library, which times every candidate
on the caller's batch with kernel-stamped events (the fused kernel alone, eager
launches of a plan) and keeps the fastest; results are cached in a text file
keyed by the batch shape and the device's compute-unit count, so a later
``tuned_plan`` for the same shape costs one file read.  Tuning plans write their
own outputs; the caller's state, controls and counters are only read.  This
module only marshals arguments.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
import torch

from . import _lib as L
from . import core

DEFAULT_CACHE = os.environ.get("SMPPI_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "smppi", "autotune.txt"))
KEYS = ("pipeline", "block", "tile", "grid")


@dataclass
class TuneResult:
    key: str
    best: Dict[str, int]
    best_ms: float
    table: List[dict] = field(default_factory=list)
    cached: bool = False


def _n_cu(ctx: core.Context) -> int:
    return torch.cuda.get_device_properties(ctx.device).multi_processor_count


def _entry(d: dict) -> L.TuneEntry:
    return L.TuneEntry(int(d["pipeline"]), int(d["block"]), int(d["tile"]), int(d["grid"]), 0.0)


def _dict(e: L.TuneEntry) -> dict:
    return {k: int(getattr(e, k)) for k in KEYS}


def shape_key(db, n_cu: int) -> str:
    """Batch shape signature (smppi_autotune_key): B, total samples to 1/8 octave,
    largest K and T, mean T, obstacles present, compute units."""
    k_off = np.ascontiguousarray(np.concatenate([[0], np.cumsum(np.asarray(db.K, dtype=np.int64))]), dtype=np.int64)
    t_off = np.ascontiguousarray(np.concatenate([[0], np.cumsum(np.asarray(db.T, dtype=np.int64))]), dtype=np.int32)
    buf = ctypes.create_string_buffer(256)
    st = L.lib().smppi_autotune_key(int(db.B), k_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    t_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    int(db.track.obs_max > 0), int(n_cu), buf, len(buf))
    if st != 0:
        raise L.SmppiError(st, "smppi_autotune_key")
    return buf.value.decode()


def candidates(n_cu: int) -> List[Dict[str, int]]:
    """The default candidate set (smppi_autotune_candidates)."""
    n = L.lib().smppi_autotune_candidates(int(n_cu), None, 0)
    arr = (L.TuneEntry * n)()
    L.lib().smppi_autotune_candidates(int(n_cu), arr, n)
    return [_dict(e) for e in arr]


def tune(ctx: core.Context, db: core.DeviceBatch, model: dict, cost: dict, seed: int, lam: float, *,
         cands: Optional[List[Dict[str, int]]] = None, reps: int = 5, warmup: int = 2,
         cache: Optional[str] = DEFAULT_CACHE, force: bool = False) -> TuneResult:
    """Time each candidate geometry on this batch; return the fastest (and the table).

    With a cache path, a stored result for the same shape key is returned without
    timing unless ``force``; a new result replaces that key's line in the file."""
    if db.dtype != torch.float32:
        raise ValueError("plans run in FP32")
    n_cu = _n_cu(ctx)
    key = shape_key(db, n_cu)
    if cache:
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
    S, V_plus = db.new_S(), db.new_V()
    stats = torch.empty(4 * db.B, dtype=db.dtype, device=db.device)
    bufs = L.PlanBuffers(db.x0.data_ptr(), db.V.data_ptr(), db.iter.data_ptr(), S.data_ptr(), V_plus.data_ptr(),
                         stats.data_ptr(), None)
    cl = list(cands) if cands is not None else candidates(n_cu)
    carr = (L.TuneEntry * len(cl))(*[_entry(c) for c in cl])
    table = (L.TuneEntry * len(cl))()
    best, cached, n_table = L.TuneEntry(), ctypes.c_int32(0), ctypes.c_int32(0)
    torch.cuda.synchronize()
    st = L.lib().smppi_autotune(ctx.h, ctypes.byref(db.batch), ctypes.byref(L.model_struct(model)),
                                ctypes.byref(L.cost_struct(cost)), ctypes.byref(core._noise(seed, False)),
                                ctypes.byref(db.track), float(lam), ctypes.byref(bufs), carr, len(cl), int(reps),
                                int(warmup), cache.encode() if cache else None, 1 if force else 0, ctypes.byref(best),
                                ctypes.byref(cached), table, len(cl), ctypes.byref(n_table),
                                ctypes.c_void_p(core._stream()))
    ctx.check(st, "smppi_autotune")
    steps = int(sum(k * t for k, t in zip(db.K, db.T)))
    rows = []
    for e in table[: min(n_table.value, len(cl))]:
        ms = float(e.kernel_ms)
        rows.append(dict(_dict(e), kernel_ms=ms, rollout_steps_per_s=steps / (ms * 1e-3) if ms > 0 else None))
    return TuneResult(key, _dict(best), float(best.kernel_ms), rows, cached=bool(cached.value))


def tuned_plan(ctx: core.Context, db: core.DeviceBatch, model: dict, cost: dict, seed: int, lam: float, *,
               cache: Optional[str] = DEFAULT_CACHE, **plan_kwargs) -> core.Plan:
    """A plan with the tuned geometry for this batch shape (tuning first if the
    cache has no entry).  ``plan_kwargs`` are the other Plan options (repair,
    execute, dist, use_graph, nominal)."""
    res = tune(ctx, db, model, cost, seed, lam, cache=cache)
    return core.Plan(ctx, db, model, cost, seed, lam, **res.best, **plan_kwargs)
