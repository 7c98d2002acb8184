"""Python face of libsmppi: device-resident problem batches and thin wrappers
with the names of the C ABI (smppi_rollout -> rollout, ...).

Only argument marshalling happens here; all arithmetic of the sampled-rollout
step runs in the library's HIP kernels on the tensors' device.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from ._lib import SmppiError


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Context:
    """One library context bound to a HIP device (scratch, tickets, error flags)."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        st = L.lib().smppi_create(int(device), ctypes.byref(h))
        if st:
            raise SmppiError(st, f"smppi_create(device={device})")
        self.h = h
        self.device = device
        self._reserved = set()

    def check(self, st: int, what: str):
        if st:
            msg = L.lib().smppi_last_error(self.h)
            raise SmppiError(st, f"{what}: {msg.decode() if msg else ''}")

    def reserve(self, db: "DeviceBatch"):
        """smppi_reserve_batch for db's bounds (a host call that allocates only when the
        ctx's scratch is smaller; the calls below make it once per new batch shape)."""
        key = (db.B, db.batch.k_max, db.batch.t_max, db.batch.dtype)
        if key not in self._reserved:
            self.check(L.lib().smppi_reserve_batch(self.h, ctypes.byref(db.batch)), "smppi_reserve_batch")
            self._reserved.add(key)

    def device_errors(self) -> int:
        v = ctypes.c_uint32(0)
        self.check(L.lib().smppi_device_errors(self.h, ctypes.byref(v)), "smppi_device_errors")
        return v.value

    def close(self):
        if getattr(self, "h", None):
            L.lib().smppi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def V_to_lib(Vs: Sequence[np.ndarray]) -> np.ndarray:
    """Per-problem (T, 2) control sequences -> the library layout (steer row, throttle row)."""
    return np.concatenate([np.asarray(v, dtype=np.float64).reshape(-1, 2).T.ravel() for v in Vs])


def V_from_lib(flat, Ts: Sequence[int]):
    flat = flat.detach().cpu().numpy() if isinstance(flat, torch.Tensor) else np.asarray(flat)
    out, o = [], 0
    for T in Ts:
        out.append(flat[o:o + 2 * T].reshape(2, T).T.copy())
        o += 2 * T
    return out


class DeviceBatch:
    """B problems (workloads.Problem) packed into the library's CSR layout on the GPU."""

    def __init__(self, problems, dtype=torch.float32, device="cuda:0", pid_base: int = 0):
        self.problems = list(problems)
        self.dtype = dtype
        self.device = torch.device(device)
        B = len(self.problems)
        self.B = B
        self.K = [int(p.K) for p in self.problems]
        self.T = [int(p.T) for p in self.problems]
        dev, dt = self.device, dtype
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
        self.k_off = torch.as_tensor(np.concatenate([[0], np.cumsum(self.K)]).astype(np.int64), device=dev)
        self.t_off = torch.as_tensor(np.concatenate([[0], np.cumsum(self.T)]).astype(np.int32), device=dev)
        npoly = [len(p.track.poly) for p in self.problems]
        nobs = [len(p.track.obs) for p in self.problems]
        self.poly_off = torch.as_tensor(np.concatenate([[0], np.cumsum(npoly)]).astype(np.int32), device=dev)
        self.obs_off = torch.as_tensor(np.concatenate([[0], np.cumsum(nobs)]).astype(np.int32), device=dev)
        polys = [p.track.poly.reshape(-1, 5) for p in self.problems if len(p.track.poly)]
        self.poly = f(np.concatenate(polys).ravel() if polys else np.zeros(5))
        obs = [p.track.obs.reshape(-1, 4) for p in self.problems if len(p.track.obs)]
        self.obs = f(np.concatenate(obs).ravel() if obs else np.zeros(4))
        self.circle = f(np.concatenate([p.track.circle for p in self.problems]))
        self.half_width = f(np.array([p.track.half_width for p in self.problems]))
        self.x0 = f(np.concatenate([p.x0 for p in self.problems]))
        self.V = f(V_to_lib([p.V for p in self.problems]))
        self.iter = torch.as_tensor(np.array([p.it for p in self.problems], dtype=np.int32), device=dev)
        self.k_max = max(self.K) if B else 0
        self.t_max = max(self.T)
        windows = {p.track.window for p in self.problems}
        if len(windows) != 1:
            raise ValueError("all problems of a batch share one projection window")
        self.batch = L.Batch(B, self.k_max, self.t_max, int(pid_base), L.F32 if dtype == torch.float32 else L.F64,
                             self.k_off.data_ptr(), self.t_off.data_ptr())
        self.track = L.Track(self.poly_off.data_ptr(), self.poly.data_ptr(), self.circle.data_ptr(),
                             self.half_width.data_ptr(), self.obs_off.data_ptr(), self.obs.data_ptr(),
                             int(windows.pop()), max(npoly), max(nobs))
        self.sum_K = int(sum(self.K))
        self.sum_T = int(sum(self.T))

    # convenience ----------------------------------------------------------
    def new_S(self):
        return torch.empty(self.sum_K, dtype=self.dtype, device=self.device)

    def new_V(self):
        return torch.empty(2 * self.sum_T, dtype=self.dtype, device=self.device)

    def controls(self, V: Optional[torch.Tensor] = None):
        return V_from_lib(self.V if V is None else V, self.T)

    def per_problem(self, x: torch.Tensor):
        a = x.detach().cpu().numpy()
        return [a[self.k_off[b].item():self.k_off[b + 1].item()] for b in range(self.B)]


def _noise(seed: int, nominal: bool):
    return L.Noise(int(seed) & 0xFFFFFFFF, 1 if nominal else 0)


def rollout(ctx: Context, db: DeviceBatch, model: dict, cost: dict, seed: int, nominal: bool = False,
            V=None, x0=None, iters=None, S=None, want_eps: bool = False):
    """smppi_rollout: per-sample modified costs S~ [sum K] (and effective noise if asked)."""
    S = db.new_S() if S is None else S
    eps = torch.zeros(db.sum_K * db.t_max * 2, dtype=db.dtype, device=db.device) if want_eps else None
    ctx.reserve(db)
    st = L.lib().smppi_rollout(ctx.h, ctypes.byref(db.batch), ctypes.byref(L.model_struct(model)),
                               ctypes.byref(L.cost_struct(cost)), ctypes.byref(_noise(seed, nominal)),
                               ctypes.byref(db.track), _p(db.x0 if x0 is None else x0), _p(db.V if V is None else V),
                               _p(db.iter if iters is None else iters), _p(S), _p(eps), ctypes.c_void_p(_stream()))
    ctx.check(st, "smppi_rollout")
    return (S, eps.view(db.sum_K, db.t_max, 2)) if want_eps else S


class CurvTrackArrays:
    """Device arrays of smppi_curv_track: per-problem periodic curvature tables
    (kappa, ds) and half widths, in problem order."""

    def __init__(self, tables, half_widths, dtype=torch.float32, device="cuda"):
        f = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64), dtype=dtype, device=device)
        n = [len(k) for k, _ in tables]
        self.kappa_off = torch.as_tensor(np.concatenate([[0], np.cumsum(n)]).astype(np.int32), device=device)
        self.kappa = f(np.concatenate([np.asarray(k, dtype=np.float64) for k, _ in tables]))
        self.ds = f([d for _, d in tables])
        self.half_width = f(half_widths)
        self.n_max = max(n)
        self.track = L.CurvTrack(self.kappa_off.data_ptr(), self.kappa.data_ptr(), self.ds.data_ptr(),
                                 self.half_width.data_ptr(), int(self.n_max))


def rollout_curvilinear(ctx: Context, db: DeviceBatch, ct: CurvTrackArrays, model: dict, wheels: dict, cost: dict,
                        seed: int, nominal: bool = False, x0=None, V=None, iters=None, S=None, want_eps: bool = False):
    """smppi_rollout_curvilinear: S~ [sum K] of the eight-state curvilinear model; x0
    (default db.x0) holds (v_x, v_y, r, omega_F, omega_R, e_psi, e_y, s) per problem."""
    S = db.new_S() if S is None else S
    eps = torch.zeros(db.sum_K * db.t_max * 2, dtype=db.dtype, device=db.device) if want_eps else None
    st = L.lib().smppi_rollout_curvilinear(ctx.h, ctypes.byref(db.batch), ctypes.byref(L.model_struct(model)),
                                           ctypes.byref(L.wheels_struct(wheels)), ctypes.byref(L.cost_struct(cost)),
                                           ctypes.byref(_noise(seed, nominal)), ctypes.byref(ct.track),
                                           _p(db.x0 if x0 is None else x0), _p(db.V if V is None else V),
                                           _p(db.iter if iters is None else iters), _p(S), _p(eps),
                                           ctypes.c_void_p(_stream()))
    ctx.check(st, "smppi_rollout_curvilinear")
    return (S, eps.view(db.sum_K, db.t_max, 2)) if want_eps else S


def rollout_backward_curvilinear(ctx: Context, db: DeviceBatch, ct: CurvTrackArrays, model: dict, wheels: dict,
                                 cost: dict, seed: int, grad_S: torch.Tensor, objective: dict, nominal: bool = False,
                                 x0=None, V=None, iters=None, out=None):
    """smppi_rollout_backward_curvilinear: sum_m grad_S[m] dL_m/dV (library layout)."""
    out = db.new_V() if out is None else out
    ctx.reserve(db)
    st = L.lib().smppi_rollout_backward_curvilinear(
        ctx.h, ctypes.byref(db.batch), ctypes.byref(L.model_struct(model)), ctypes.byref(L.wheels_struct(wheels)),
        ctypes.byref(L.cost_struct(cost)), ctypes.byref(_noise(seed, nominal)), ctypes.byref(ct.track),
        _p(db.x0 if x0 is None else x0), _p(db.V if V is None else V), _p(db.iter if iters is None else iters),
        _p(grad_S), ctypes.byref(L.objective_struct(objective)), _p(out), ctypes.c_void_p(_stream()))
    ctx.check(st, "smppi_rollout_backward_curvilinear")
    return out


def shield_repair_curvilinear(ctx: Context, db: DeviceBatch, ct: CurvTrackArrays, model: dict, wheels: dict,
                              cost: dict, V_plus: torch.Tensor, n_steps: int, step: float, objective: dict, x0=None,
                              out=None):
    """smppi_shield_repair_curvilinear: Algorithm 1 on the curvilinear model."""
    out = db.new_V() if out is None else out
    opts = L.repair_opts(n_steps, step, objective, "gradient")
    st = L.lib().smppi_shield_repair_curvilinear(
        ctx.h, ctypes.byref(db.batch), ctypes.byref(L.model_struct(model)), ctypes.byref(L.wheels_struct(wheels)),
        ctypes.byref(L.cost_struct(cost)), ctypes.byref(ct.track), _p(db.x0 if x0 is None else x0), _p(V_plus),
        ctypes.byref(opts), _p(out), ctypes.c_void_p(_stream()))
    ctx.check(st, "smppi_shield_repair_curvilinear")
    return out


def execute_curvilinear(ctx: Context, db: DeviceBatch, ct: CurvTrackArrays, model: dict, wheels: dict,
                        V_exec: torch.Tensor, V_plus: torch.Tensor, dist: Optional[torch.Tensor] = None,
                        n_dist: int = 0):
    """smppi_execute_curvilinear: advances db.x0 (eight states), warm-starts db.V, increments db.iter."""
    st = L.lib().smppi_execute_curvilinear(ctx.h, ctypes.byref(db.batch), ctypes.byref(L.model_struct(model)),
                                           ctypes.byref(L.wheels_struct(wheels)), ctypes.byref(ct.track), _p(V_exec),
                                           _p(V_plus), _p(dist), int(n_dist), _p(db.x0), _p(db.V), _p(db.iter),
                                           ctypes.c_void_p(_stream()))
    ctx.check(st, "smppi_execute_curvilinear")


def weights(ctx: Context, db: DeviceBatch, S: torch.Tensor, lam: float):
    """smppi_weights: (w [sum K], stats [B][4])."""
    w = torch.empty_like(S)
    stats = torch.empty(4 * db.B, dtype=db.dtype, device=db.device)
    st = L.lib().smppi_weights(ctx.h, ctypes.byref(db.batch), _p(S), float(lam), _p(w), _p(stats),
                               ctypes.c_void_p(_stream()))
    ctx.check(st, "smppi_weights")
    return w, stats.view(db.B, 4)


def update(ctx: Context, db: DeviceBatch, model: dict, cost: dict, seed: int, w: torch.Tensor,
           nominal: bool = False, V=None, iters=None, out=None):
    """smppi_update: V+ in the library layout."""
    V = db.V if V is None else V
    out = db.new_V() if out is None else out
    ctx.reserve(db)
    st = L.lib().smppi_update(ctx.h, ctypes.byref(db.batch), ctypes.byref(L.model_struct(model)),
                              ctypes.byref(L.cost_struct(cost)), ctypes.byref(_noise(seed, nominal)), _p(V), _p(w),
                              _p(db.iter if iters is None else iters), _p(out), ctypes.c_void_p(_stream()))
    ctx.check(st, "smppi_update")
    return out


def rollout_backward(ctx: Context, db: DeviceBatch, model: dict, cost: dict, seed: int, grad_S: torch.Tensor,
                     objective: dict, nominal: bool = False, V=None, x0=None, iters=None, out=None,
                     noalloc: bool = False):
    """smppi_rollout_backward: sum_m grad_S[m] dL_m/dV in the library layout.
    noalloc=True calls smppi_rollout_backward_noalloc (fixed device scratch, nothing
    reserved or allocated; `out` should then be preallocated by the caller)."""
    V = db.V if V is None else V
    out = db.new_V() if out is None else out
    if noalloc:
        fn, name = L.lib().smppi_rollout_backward_noalloc, "smppi_rollout_backward_noalloc"
    else:
        ctx.reserve(db)
        fn, name = L.lib().smppi_rollout_backward, "smppi_rollout_backward"
    st = fn(
        ctx.h, ctypes.byref(db.batch), ctypes.byref(L.model_struct(model)), ctypes.byref(L.cost_struct(cost)),
        ctypes.byref(_noise(seed, nominal)), ctypes.byref(db.track), _p(db.x0 if x0 is None else x0), _p(V),
        _p(db.iter if iters is None else iters), _p(grad_S), ctypes.byref(L.objective_struct(objective)), _p(out),
        ctypes.c_void_p(_stream()))
    ctx.check(st, name)
    return out


def shield_repair(ctx: Context, db: DeviceBatch, model: dict, cost: dict, V_plus: torch.Tensor, n_steps: int,
                  step: float, objective: dict, x0=None, out=None, method: str = "gradient", memory: int = 5):
    """smppi_shield_repair: V_safe in the library layout (method "gradient": Algorithm 1;
    "lbfgs": projected L-BFGS with `memory` pairs)."""
    out = db.new_V() if out is None else out
    opts = L.repair_opts(n_steps, step, objective, method, memory)
    st = L.lib().smppi_shield_repair(ctx.h, ctypes.byref(db.batch), ctypes.byref(L.model_struct(model)),
                                     ctypes.byref(L.cost_struct(cost)), ctypes.byref(db.track),
                                     _p(db.x0 if x0 is None else x0), _p(V_plus), ctypes.byref(opts), _p(out),
                                     ctypes.c_void_p(_stream()))
    ctx.check(st, "smppi_shield_repair")
    return out


def execute(ctx: Context, db: DeviceBatch, model: dict, V_exec: torch.Tensor, V_plus: torch.Tensor,
            dist: Optional[torch.Tensor] = None, n_dist: int = 0, x=None, V=None, iters=None):
    """smppi_execute: advance the plant state and warm-start V in place (defaults: the batch's own)."""
    st = L.lib().smppi_execute(ctx.h, ctypes.byref(db.batch), ctypes.byref(L.model_struct(model)), _p(V_exec),
                               _p(V_plus), _p(dist), int(n_dist), _p(db.x0 if x is None else x),
                               _p(db.V if V is None else V), _p(db.iter if iters is None else iters),
                               ctypes.c_void_p(_stream()))
    ctx.check(st, "smppi_execute")


class Plan:
    """smppi_plan_*: the persistent fused launch (+ shield, + execute), optionally in a HIP graph.

    Reads db.x0 / db.V / db.iter and writes S, V_plus, stats (and V_safe); with
    execute=True it advances db.x0, db.V and db.iter in place, so repeated
    launches run the closed loop on the device."""

    def __init__(self, ctx: Context, db: DeviceBatch, model: dict, cost: dict, seed: int, lam: float,
                 repair: Optional[dict] = None, execute: bool = False, dist: Optional[torch.Tensor] = None,
                 block: int = 0, tile: int = 0, grid: int = 0, use_graph: bool = True, nominal: bool = False,
                 pipeline: int = 0, fuse_shield: int = 0):
        if db.dtype != torch.float32:
            raise ValueError("plans run in FP32")
        self.ctx, self.db = ctx, db
        self.S = db.new_S()
        self.V_plus = db.new_V()
        self.V_safe = db.new_V() if repair else None
        self.stats = torch.empty(4 * db.B, dtype=db.dtype, device=db.device)
        self.dist = dist
        ro = L.RepairOpts(0, 0.0, L.Objective(0, 0, 0, 0), 0, 0)
        if repair:
            ro = L.repair_opts(repair["n_steps"], repair["step"], repair["objective"],
                               repair.get("method", "gradient"), repair.get("memory", 5))
        opts = L.PlanOpts(float(lam), 1 if repair else 0, ro, 1 if execute else 0,
                          dist.data_ptr() if dist is not None else None,
                          int(dist.shape[0]) if dist is not None else 0, int(block), int(tile), int(grid),
                          1 if use_graph else 0, int(pipeline), int(fuse_shield))
        bufs = L.PlanBuffers(db.x0.data_ptr(), db.V.data_ptr(), db.iter.data_ptr(), self.S.data_ptr(),
                             self.V_plus.data_ptr(), self.stats.data_ptr(),
                             self.V_safe.data_ptr() if self.V_safe is not None else None)
        self._keep = (opts, bufs)
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        st = L.lib().smppi_plan_create(ctx.h, ctypes.byref(db.batch), ctypes.byref(L.model_struct(model)),
                                       ctypes.byref(L.cost_struct(cost)), ctypes.byref(_noise(seed, nominal)),
                                       ctypes.byref(db.track), ctypes.byref(opts), ctypes.byref(bufs),
                                       ctypes.byref(h))
        ctx.check(st, "smppi_plan_create")
        self.h = h

    def launch(self):
        self.ctx.check(L.lib().smppi_plan_launch(self.h, ctypes.c_void_p(_stream())), "smppi_plan_launch")

    def launch_profiled(self):
        self.ctx.check(L.lib().smppi_plan_launch_profiled(self.h, ctypes.c_void_p(_stream())),
                       "smppi_plan_launch_profiled")

    def stage_ms(self):
        """(fused, repair, execute) durations in ms of the last profiled launch."""
        f, r, e = ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
        self.ctx.check(L.lib().smppi_plan_stage_ms(self.h, ctypes.byref(f), ctypes.byref(r), ctypes.byref(e)),
                       "smppi_plan_stage_ms")
        return f.value, r.value, e.value

    def kernel_ms(self):
        """(fused kernel, shield kernel) durations in ms of the last profiled launch,
        from events stamped with the kernels' own start and end."""
        f, r = ctypes.c_float(), ctypes.c_float()
        self.ctx.check(L.lib().smppi_plan_kernel_ms(self.h, ctypes.byref(f), ctypes.byref(r)),
                       "smppi_plan_kernel_ms")
        return f.value, r.value

    def info(self):
        g, b, t, n = (ctypes.c_int32() for _ in range(4))
        self.ctx.check(L.lib().smppi_plan_info(self.h, ctypes.byref(g), ctypes.byref(b), ctypes.byref(t),
                                               ctypes.byref(n)), "smppi_plan_info")
        return dict(grid=g.value, block=b.value, tile=t.value, n_tiles=n.value)

    def close(self):
        if getattr(self, "h", None):
            L.lib().smppi_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_philox(ctx: Context, ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x32-10 words computed by the device generator for counters ctr [n][4]."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    n = ctr.shape[0]
    dc = torch.as_tensor(ctr.view(np.int32), device=f"cuda:{ctx.device}")
    out = torch.empty_like(dc)
    k = (ctypes.c_uint32 * 2)(int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF)
    st = L.lib().smppi_debug_philox(ctx.h, _p(dc), k, n, _p(out), ctypes.c_void_p(_stream()))
    ctx.check(st, "smppi_debug_philox")
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)
