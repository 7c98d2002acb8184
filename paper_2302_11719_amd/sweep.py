"""Closed-loop collision sweep: the paper's second experiment (Sec. VI-E, the
collision-rate comparison over sample count and horizon of Figs. 5 and 6) made
device-resident and batched, on generated tracks.

For every (K, T) cell and controller, `runs` independent closed loops (one
problem each: its own spline track, start speed and disturbance sequence) run
`steps` receding-horizon iterations through one batched plan: the fused
rollout/weights/update launch, the shield when the controller has it, and the
disturbed plant step of eq. (26), all on the device.  After every iteration the
executed states are checked against the track boundary and the obstacles; the
collision rate of a cell is the fraction of runs that left the safe set at least
once.

Controllers:
  "mppi"       MPPI with the state cost of eq. (24) and the collision indicator
               of eq. (25), no barrier penalty (C_cbf = 0), no shield;
  "mppi_dcbf"  the same plus the DCBF penalty of eqs. (17)-(20) in the sampled cost;
  "shield"     Shield-MPPI: the DCBF cost and the shield of Algorithm 1 (or its
               L-BFGS variant).

The absolute rates are those of this model and these synthetic tracks, not the
paper's vehicle and track.
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import Dict, Iterable, List, Optional

import numpy as np
import torch

from . import core
from . import workloads as W

CONTROLLERS = ("mppi", "mppi_dcbf", "shield")


def segment_distance_sq(poly: np.ndarray, p: np.ndarray) -> np.ndarray:
    """Squared distance from points p [n][2] to the nearest segment of a closed
    polyline given as rows (a_x, a_y, d_x, d_y, 1/|d|^2)."""
    a = poly[None, :, 0:2]
    dv = poly[None, :, 2:4]
    r = p[:, None, :] - a
    lam = np.clip((r * dv).sum(-1) * poly[None, :, 4], 0.0, 1.0)
    e = r - lam[..., None] * dv
    return (e * e).sum(-1).min(axis=1)


def collided(track: W.Track, p: np.ndarray) -> np.ndarray:
    """Whether points p [n][2] lie outside the track (|e_y| > half width) or inside
    an obstacle (distance < radius)."""
    if track.kind == 0:
        cx, cy, R = track.circle
        e2 = (np.hypot(p[:, 0] - cx, p[:, 1] - cy) - R) ** 2
    else:
        e2 = segment_distance_sq(track.poly, p)
    out = e2 > track.half_width ** 2
    if len(track.obs):
        o = np.asarray(track.obs)
        d2 = (p[:, None, 0] - o[None, :, 0]) ** 2 + (p[:, None, 1] - o[None, :, 1]) ** 2
        out = out | (d2 < o[None, :, 3]).any(axis=1)
    return out


@dataclass
class Cell:
    K: int
    T: int
    controller: str
    runs: int
    steps: int
    collision_rate: float
    collisions_per_run: float
    ms_per_step: float


def batch_collided(tracks: List[W.Track], p: np.ndarray) -> np.ndarray:
    """collided() for one point per track, p [runs][2]; polylines of equal length
    are evaluated together."""
    if all(t.kind == 1 for t in tracks) and len({len(t.poly) for t in tracks}) == 1 and not any(
            len(t.obs) for t in tracks):
        poly = np.stack([t.poly for t in tracks])                      # [R][N][5]
        r = p[:, None, :] - poly[:, :, 0:2]
        lam = np.clip((r * poly[:, :, 2:4]).sum(-1) * poly[:, :, 4], 0.0, 1.0)
        e = r - lam[..., None] * poly[:, :, 2:4]
        e2 = (e * e).sum(-1).min(axis=1)
        return e2 > np.array([t.half_width for t in tracks]) ** 2
    return np.array([collided(t, p[i:i + 1])[0] for i, t in enumerate(tracks)])


def make_runs(runs: int, K: int, T: int, seed: int = 0, n_obs: int = 0, half_width: float = 0.9) -> List[W.Problem]:
    """One problem per run: spline track seed + run, start speed U[2, 4] m/s,
    zero initial controls; obstacles when n_obs > 0."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(runs):
        tr = W.spline_track(seed * 100000 + r, half_width=half_width)
        if n_obs:
            tr.obs = W.obstacles(tr, seed * 100000 + r, n=n_obs)
        x0 = W.start_state(tr, vx=float(rng.uniform(2.0, 4.0)))
        out.append(W.round_to_f32(W.Problem(K, T, tr, x0, np.zeros((T, 2)), r, 0)))
    return out


@dataclass
class CellSetup:
    """The device objects of one cell: its plan (closed loop on the device), batch,
    problems, model and cost constants (FP32-rounded), disturbances [steps][runs][2]
    and shield options (None without the shield)."""
    plan: core.Plan
    db: core.DeviceBatch
    probs: List[W.Problem]
    model: dict
    cost: dict
    dist: np.ndarray
    repair: Optional[dict]
    seed: int
    lam: float


def setup_cell(ctx: core.Context, K: int, T: int, controller: str, runs: int, steps: int, seed: int = 0,
               n_obs: int = 0, dist_sigma: float = 0.3, lam: float = W.LAMBDA, repair: Optional[dict] = None,
               v_goal: Optional[float] = None, half_width: float = 0.9, use_graph: bool = True) -> CellSetup:
    """Builds one (K, T, controller) cell: `runs` problems and the plan that advances
    all of them by one receding-horizon step per launch."""
    if controller not in CONTROLLERS:
        raise ValueError(controller)
    cost = dict(W.COST)
    if controller == "mppi":
        cost["C_cbf"] = 0.0
    if v_goal is not None:
        cost["v_g"] = float(v_goal)
    M, C = W.params_f32(W.MODEL, cost)
    probs = make_runs(runs, K, T, seed, n_obs, half_width)
    db = core.DeviceBatch(probs, dtype=torch.float32)
    dist = W.disturbances(seed + 17, steps * runs, sigma=dist_sigma).reshape(steps, runs, 2).astype(np.float32)
    dist_t = torch.as_tensor(dist, device="cuda")
    rep = None
    if controller == "shield":
        rep = repair or dict(n_steps=10, step=0.05, objective=W.OBJ_SHIELD)
    plan = core.Plan(ctx, db, M, C, seed, lam, repair=rep, execute=True, dist=dist_t, use_graph=use_graph)
    plan._dist_keep = dist_t
    return CellSetup(plan, db, probs, M, C, dist, rep, seed, lam)


def run_cell(ctx: core.Context, K: int, T: int, controller: str, runs: int = 100, steps: int = 100,
             seed: int = 0, n_obs: int = 0, dist_sigma: float = 0.3, lam: float = W.LAMBDA,
             repair: Optional[dict] = None, v_goal: Optional[float] = None, half_width: float = 0.9) -> Cell:
    """One (K, T, controller) cell of the sweep (v_goal: target speed of the state
    cost, default the workload's)."""
    cs = setup_cell(ctx, K, T, controller, runs, steps, seed, n_obs, dist_sigma, lam, repair, v_goal, half_width)
    plan, db, probs = cs.plan, cs.db, cs.probs
    tracks = [p.track for p in probs]
    hit = np.zeros(runs, dtype=bool)
    count = np.zeros(runs, dtype=np.int64)
    t_gpu = 0.0
    for _ in range(steps):
        t0 = time.perf_counter()
        plan.launch()
        x = db.x0.view(runs, 6)[:, :2].cpu().numpy().astype(np.float64)  # synchronises
        t_gpu += time.perf_counter() - t0
        c = batch_collided(tracks, x)
        hit |= c
        count += c
    plan.close()
    return Cell(K, T, controller, runs, steps, float(hit.mean()), float(count.mean()), 1e3 * t_gpu / steps)


def sweep(ctx: core.Context, Ks: Iterable[int], Ts: Iterable[int], controllers: Iterable[str] = CONTROLLERS,
          runs: int = 100, steps: int = 100, seed: int = 0, **kw) -> List[Dict]:
    """Collision rate for every (K, T, controller) cell (kw: run_cell options)."""
    rows = []
    for K in Ks:
        for T in Ts:
            for c in controllers:
                rows.append(run_cell(ctx, K, T, c, runs, steps, seed, **kw).__dict__)
    return rows
