"""FP64 CPU oracle of the Shield-MPPI sampled-rollout step (arXiv 2302.11719).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The product library never imports
or links it, and it imports nothing from the product package: inputs arrive as
plain numpy arrays and parameter dicts.

The arithmetic lives in ``smppi_oracle.cpp`` (plain scalar C++17, FP64, no
contraction).  This module only marshals arguments.  Control sequences here are
``[T][2]`` (time major); the GPU library's ``[2][T]`` layout is converted by the
tests.

Section/equation map (paper):
  * noise: Section II (u ~ N(v, Sigma)), Algorithm 2 sampling step;
  * dynamics: eq. (1) realised as a six-state single-track model, RK4;
  * barrier: eq. (23) track barrier, plus circular obstacle barriers;
  * cost: eqs. (8), (12), (17)-(20), (24), (25), Algorithm 2;
  * weights: eqs. (7), (9), (11);  update: eq. (10);
  * repair: eq. (22) and Algorithm 1 (projected gradient steps);
  * closed loop: Algorithm 2 outer loop with the disturbed plant of eq. (26).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "smppi_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_ABI = 7
_lock = threading.Lock()
_lib = None

MODEL_KEYS = ("m", "lf", "lr", "Iz", "Cf", "Cr", "a_max", "c_v", "v_min", "dt")
COST_KEYS = ("v_g", "q_v", "q_ey", "C_obs", "phi_w", "lambda_u", "sigma0", "sigma1", "C_cbf", "gamma")


def build(force: bool = False) -> str:
    """Compile liboracle.so with g++ (scalar FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-pthread", _SRC, "-o", _LIB + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            if L.or_abi_version() != _ABI:
                build(force=True)
                raise RuntimeError("stale liboracle.so was rebuilt; restart the process")
            L.or_lateral_sq.restype = ctypes.c_double
            L.or_objective.restype = ctypes.c_double
            L.or_objective_c8.restype = ctypes.c_double
            L.or_kappa_at.restype = ctypes.c_double
            _lib = L
    return _lib


def _p(a, dtype=np.float64):
    if a is None:
        return None
    return np.ascontiguousarray(a, dtype=dtype).ctypes.data_as(ctypes.c_void_p)


def model_array(model: dict) -> np.ndarray:
    return np.array([model[k] for k in MODEL_KEYS] + list(model["u_lo"]) + list(model["u_hi"]),
                    dtype=np.float64)


def cost_array(cost: dict) -> np.ndarray:
    c = dict(cost)
    c["sigma0"], c["sigma1"] = cost["sigma"]
    return np.array([c[k] for k in COST_KEYS], dtype=np.float64)


class _TrackArgs:
    """Keeps the contiguous arrays of one track alive while a call runs."""

    def __init__(self, track):
        self.kind = int(track.kind)
        self.circle = np.ascontiguousarray(track.circle, dtype=np.float64)
        self.poly = np.ascontiguousarray(track.poly, dtype=np.float64).reshape(-1, 5)
        self.obs = np.ascontiguousarray(track.obs, dtype=np.float64).reshape(-1, 4)
        self.w = float(track.half_width)
        self.window = int(track.window)

    def args(self):
        return (ctypes.c_int(self.kind), _p(self.circle), _p(self.poly) if len(self.poly) else None,
                ctypes.c_int(len(self.poly)), ctypes.c_double(self.w),
                _p(self.obs) if len(self.obs) else None, ctypes.c_int(len(self.obs)),
                ctypes.c_int(self.window))


# --------------------------------------------------------------------------- noise
def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox(_p(c, np.uint32), _p(k, np.uint32), _p(out, np.uint32))
    return out


def normals(seed: int, pid: int, it: int, m: int, T: int) -> np.ndarray:
    """Standard normals [T][2] of sample m (before scaling by sigma)."""
    z = np.zeros((T, 2))
    lib().or_normals(ctypes.c_uint32(seed), ctypes.c_uint32(pid), ctypes.c_uint32(it), ctypes.c_uint32(m),
                     ctypes.c_int(T), _p(z))
    return z


# --------------------------------------------------------------------------- dynamics
def deriv(model: dict, x, u) -> np.ndarray:
    out = np.zeros(6)
    mp = model_array(model)
    lib().or_deriv(_p(mp), _p(x), _p(u), _p(out))
    return out


def rk4(model: dict, x, u, dt: float, n_steps: int = 1) -> np.ndarray:
    out = np.zeros(6)
    mp = model_array(model)
    lib().or_rk4(_p(mp), _p(x), _p(u), ctypes.c_double(dt), ctypes.c_int(n_steps), _p(out))
    return out


def lateral_sq(track, px: float, py: float, idx: int = -1):
    """(e_y^2, chosen segment): global search when idx < 0, else the window rule."""
    ta = _TrackArgs(track)
    out = ctypes.c_int(0)
    e2 = lib().or_lateral_sq(ctypes.c_int(ta.kind), _p(ta.circle), _p(ta.poly) if len(ta.poly) else None,
                             ctypes.c_int(len(ta.poly)), ctypes.c_int(ta.window), ctypes.c_double(px),
                             ctypes.c_double(py), ctypes.c_int(idx), ctypes.byref(out))
    return e2, out.value


# --------------------------------------------------------------------------- MPPI step
def rollout(model, cost, track, x0, V, K: int, seed: int, pid: int, it: int, nominal: bool = False,
            want_eps: bool = True, n_threads: int = 1, samples=None):
    """Per-sample modified costs S~ [K], effective noise eps' [K][T][2], indicator margins [K].
    With `samples` (sample indices), evaluates just those samples (K is ignored)."""
    V = np.ascontiguousarray(V, dtype=np.float64).reshape(-1, 2)
    ms = None
    if samples is not None:
        ms = np.ascontiguousarray(samples, dtype=np.uint32)
        K = len(ms)
    T = V.shape[0]
    S = np.zeros(K)
    margin = np.zeros(K)
    eps = np.zeros((K, T, 2)) if want_eps else None
    mp, cp, ta = model_array(model), cost_array(cost), _TrackArgs(track)
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    lib().or_rollout(_p(mp), _p(cp), *ta.args(), _p(x0), _p(V), ctypes.c_int(K), ctypes.c_int(T),
                     ctypes.c_uint32(seed), ctypes.c_uint32(pid), ctypes.c_uint32(it), ctypes.c_int(int(nominal)),
                     _p(ms, np.uint32) if ms is not None else None, _p(S), _p(eps) if want_eps else None,
                     _p(margin), ctypes.c_int(n_threads))
    return S, eps, margin


def weights(S, lam: float):
    """(w [K], stats [S_min, log sum omega, ESS, n_nonfinite])."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    w = np.zeros_like(S)
    stats = np.zeros(4)
    lib().or_weights(_p(S), ctypes.c_int(len(S)), ctypes.c_double(lam), _p(w), _p(stats))
    return w, stats


def update(V, w, eps_eff) -> np.ndarray:
    V = np.ascontiguousarray(V, dtype=np.float64).reshape(-1, 2)
    eps_eff = np.ascontiguousarray(eps_eff, dtype=np.float64)
    K, T = eps_eff.shape[0], eps_eff.shape[1]
    Vp = np.zeros_like(V)
    lib().or_update(_p(V), _p(w), _p(eps_eff), ctypes.c_int(K), ctypes.c_int(T), _p(Vp))
    return Vp


def mppi_iteration(model, cost, track, x0, V, K, seed, pid, it, lam, nominal=False, n_threads=1):
    """One sampling + weighting + update pass (Algorithm 2 without the shield)."""
    S, eps, margin = rollout(model, cost, track, x0, V, K, seed, pid, it, nominal, True, n_threads)
    w, stats = weights(S, lam)
    Vp = update(V, w, eps)
    return dict(S=S, eps=eps, margin=margin, w=w, stats=stats, V_plus=Vp)


# --------------------------------------------------------------------------- gradients and repair
def _objective_args(obj):
    return (ctypes.c_double(obj["w_S"]), ctypes.c_double(obj["w_sq"]), ctypes.c_double(obj["w_lin"]),
            ctypes.c_int(int(obj["n_lin"])))


def objective(model, cost, track, x0, V, obj, eps=None):
    """(L, decision signature) of one trajectory; eps [T][2] raw noise or None (nominal)."""
    V = np.ascontiguousarray(V, dtype=np.float64).reshape(-1, 2)
    mp, cp, ta = model_array(model), cost_array(cost), _TrackArgs(track)
    sig = ctypes.c_uint64(0)
    L = lib().or_objective(_p(mp), _p(cp), *ta.args(), _p(x0), _p(V), ctypes.c_int(V.shape[0]),
                           _p(eps) if eps is not None else None, *_objective_args(obj), ctypes.byref(sig))
    return L, sig.value


def gradient_dual(model, cost, track, x0, V, obj, eps=None) -> np.ndarray:
    V = np.ascontiguousarray(V, dtype=np.float64).reshape(-1, 2)
    g = np.zeros_like(V)
    mp, cp, ta = model_array(model), cost_array(cost), _TrackArgs(track)
    lib().or_gradient_dual(_p(mp), _p(cp), *ta.args(), _p(x0), _p(V), ctypes.c_int(V.shape[0]),
                           _p(eps) if eps is not None else None, *_objective_args(obj), _p(g))
    return g


def gradient_fd(model, cost, track, x0, V, obj, eps=None, h: float = 1e-6):
    """(central-difference gradient, validity mask: no decision switches inside the stencil)."""
    V = np.ascontiguousarray(V, dtype=np.float64).reshape(-1, 2)
    g = np.zeros_like(V)
    valid = np.zeros(V.shape, dtype=np.int32)
    mp, cp, ta = model_array(model), cost_array(cost), _TrackArgs(track)
    lib().or_gradient_fd(_p(mp), _p(cp), *ta.args(), _p(x0), _p(V), ctypes.c_int(V.shape[0]),
                         _p(eps) if eps is not None else None, *_objective_args(obj), ctypes.c_double(h),
                         _p(g), _p(valid, np.int32))
    return g, valid.astype(bool)


def repair(model, cost, track, x0, V_plus, n_steps: int, step: float, obj, method: str = "gradient",
           memory: int = 5) -> np.ndarray:
    """Safety shield: Algorithm 1 (method "gradient") or the projected L-BFGS
    variant ("lbfgs", `memory` pairs).  V_plus: [T][2]."""
    V_plus = np.ascontiguousarray(V_plus, dtype=np.float64).reshape(-1, 2)
    out = np.zeros_like(V_plus)
    mp, cp, ta = model_array(model), cost_array(cost), _TrackArgs(track)
    if method == "gradient":
        lib().or_repair(_p(mp), _p(cp), *ta.args(), _p(x0), _p(V_plus), ctypes.c_int(V_plus.shape[0]),
                        ctypes.c_int(n_steps), ctypes.c_double(step), *_objective_args(obj), _p(out))
    elif method == "lbfgs":
        lib().or_repair_lbfgs(_p(mp), _p(cp), *ta.args(), _p(x0), _p(V_plus), ctypes.c_int(V_plus.shape[0]),
                              ctypes.c_int(n_steps), ctypes.c_double(step), *_objective_args(obj),
                              ctypes.c_int(memory), _p(out))
    else:
        raise ValueError(method)
    return out


def lbfgs_direction(g, S, Y, gamma: float) -> np.ndarray:
    """d = -H g by the two-loop recursion; S, Y: [n_pairs][n], oldest first."""
    g = np.ascontiguousarray(g, dtype=np.float64).ravel()
    S = np.ascontiguousarray(S, dtype=np.float64).reshape(-1, g.size)
    Y = np.ascontiguousarray(Y, dtype=np.float64).reshape(-1, g.size)
    d = np.zeros_like(g)
    lib().or_lbfgs_direction(_p(g), _p(S) if len(S) else None, _p(Y) if len(Y) else None, ctypes.c_int(len(S)),
                             ctypes.c_int(g.size), ctypes.c_double(gamma), _p(d))
    return d


WHEEL_KEYS = ("r_w", "I_w", "C_x")


def wheels_array(wheels: dict) -> np.ndarray:
    return np.array([wheels[k] for k in WHEEL_KEYS], dtype=np.float64)


class _CurvArgs:
    """Contiguous arrays of one curvilinear track: periodic curvature table, spacing, half width."""

    def __init__(self, kappa, ds: float, half_width: float = 0.0):
        self.kappa = np.ascontiguousarray(kappa, dtype=np.float64)
        self.ds = float(ds)
        self.w = float(half_width)

    def args(self):
        return (_p(self.kappa), ctypes.c_int(len(self.kappa)), ctypes.c_double(self.ds))


def deriv_c8(model, wheels, kappa, ds: float, x, u) -> np.ndarray:
    """f of the eight-state curvilinear model; x = (v_x, v_y, r, omega_F, omega_R, e_psi, e_y, s)."""
    out = np.zeros(8)
    ca = _CurvArgs(kappa, ds)
    lib().or_deriv_c8(_p(model_array(model)), _p(wheels_array(wheels)), *ca.args(),
                      _p(np.ascontiguousarray(x, dtype=np.float64)), _p(np.ascontiguousarray(u, dtype=np.float64)),
                      _p(out))
    return out


def rollout_c8(model, wheels, cost, kappa, ds: float, half_width: float, x0, V, K: int, seed: int, pid: int, it: int,
               nominal: bool = False, want_eps: bool = True, n_threads: int = 1):
    """Eight-state curvilinear model: per-sample S~ [K], effective noise [K][T][2], indicator margins [K]."""
    V = np.ascontiguousarray(V, dtype=np.float64).reshape(-1, 2)
    T = V.shape[0]
    ca = _CurvArgs(kappa, ds, half_width)
    S, margin = np.zeros(K), np.zeros(K)
    eps = np.zeros((K, T, 2)) if want_eps else None
    lib().or_rollout_c8(_p(model_array(model)), _p(wheels_array(wheels)), _p(cost_array(cost)), *ca.args(),
                        ctypes.c_double(ca.w), _p(np.ascontiguousarray(x0, dtype=np.float64)), _p(V), ctypes.c_int(K),
                        ctypes.c_int(T), ctypes.c_uint32(seed), ctypes.c_uint32(pid), ctypes.c_uint32(it),
                        ctypes.c_int(int(nominal)), _p(S), _p(eps) if want_eps else None, _p(margin),
                        ctypes.c_int(n_threads))
    return S, eps, margin


def trajectory_c8(model, wheels, kappa, ds: float, x0, V, eps=None) -> np.ndarray:
    """States [T+1][8] of the eight-state curvilinear model under V (+ raw noise eps [T][2])."""
    V = np.ascontiguousarray(V, dtype=np.float64).reshape(-1, 2)
    ca = _CurvArgs(kappa, ds)
    xs = np.zeros((V.shape[0] + 1, 8))
    lib().or_trajectory_c8(_p(model_array(model)), _p(wheels_array(wheels)), *ca.args(),
                           _p(np.ascontiguousarray(x0, dtype=np.float64)), _p(V), ctypes.c_int(V.shape[0]),
                           _p(eps) if eps is not None else None, _p(xs))
    return xs


def objective_c8(model, wheels, cost, kappa, ds: float, half_width: float, x0, V, obj, eps=None):
    """(L, decision signature) of one curvilinear trajectory."""
    V = np.ascontiguousarray(V, dtype=np.float64).reshape(-1, 2)
    ca = _CurvArgs(kappa, ds, half_width)
    sig = ctypes.c_uint64(0)
    L = lib().or_objective_c8(_p(model_array(model)), _p(wheels_array(wheels)), _p(cost_array(cost)), *ca.args(),
                              ctypes.c_double(ca.w), _p(np.ascontiguousarray(x0, dtype=np.float64)), _p(V),
                              ctypes.c_int(V.shape[0]), _p(eps) if eps is not None else None, *_objective_args(obj),
                              ctypes.byref(sig))
    return L, sig.value


def gradient_dual_c8(model, wheels, cost, kappa, ds: float, half_width: float, x0, V, obj, eps=None) -> np.ndarray:
    V = np.ascontiguousarray(V, dtype=np.float64).reshape(-1, 2)
    ca = _CurvArgs(kappa, ds, half_width)
    g = np.zeros_like(V)
    lib().or_gradient_dual_c8(_p(model_array(model)), _p(wheels_array(wheels)), _p(cost_array(cost)), *ca.args(),
                              ctypes.c_double(ca.w), _p(np.ascontiguousarray(x0, dtype=np.float64)), _p(V),
                              ctypes.c_int(V.shape[0]), _p(eps) if eps is not None else None, *_objective_args(obj),
                              _p(g))
    return g


def gradient_fd_c8(model, wheels, cost, kappa, ds: float, half_width: float, x0, V, obj, eps=None, h: float = 1e-6):
    V = np.ascontiguousarray(V, dtype=np.float64).reshape(-1, 2)
    ca = _CurvArgs(kappa, ds, half_width)
    g = np.zeros_like(V)
    valid = np.zeros(V.shape, dtype=np.int32)
    lib().or_gradient_fd_c8(_p(model_array(model)), _p(wheels_array(wheels)), _p(cost_array(cost)), *ca.args(),
                            ctypes.c_double(ca.w), _p(np.ascontiguousarray(x0, dtype=np.float64)), _p(V),
                            ctypes.c_int(V.shape[0]), _p(eps) if eps is not None else None, *_objective_args(obj),
                            ctypes.c_double(h), _p(g), _p(valid, np.int32))
    return g, valid.astype(bool)


def repair_c8(model, wheels, cost, kappa, ds: float, half_width: float, x0, V_plus, n_steps: int, step: float,
              obj) -> np.ndarray:
    """Algorithm 1 on the eight-state curvilinear model; V_plus [T][2]."""
    V_plus = np.ascontiguousarray(V_plus, dtype=np.float64).reshape(-1, 2)
    ca = _CurvArgs(kappa, ds, half_width)
    out = np.zeros_like(V_plus)
    lib().or_repair_c8(_p(model_array(model)), _p(wheels_array(wheels)), _p(cost_array(cost)), *ca.args(),
                       ctypes.c_double(ca.w), _p(np.ascontiguousarray(x0, dtype=np.float64)), _p(V_plus),
                       ctypes.c_int(V_plus.shape[0]), ctypes.c_int(n_steps), ctypes.c_double(step),
                       *_objective_args(obj), _p(out))
    return out


def execute_c8(model, wheels, kappa, ds: float, x, u0, dist=None) -> np.ndarray:
    """Disturbed plant step of the curvilinear model: x+ = f(x, clip(u0)) + w, w on (v_y, r)."""
    u0 = np.clip(np.asarray(u0, dtype=np.float64), model["u_lo"], model["u_hi"])
    xn = trajectory_c8(model, wheels, kappa, ds, x, u0.reshape(1, 2))[1].copy()
    if dist is not None:
        xn[1] += dist[0]
        xn[2] += dist[1]
    return xn


def kappa_at(kappa, ds: float, s: float) -> float:
    kappa = np.ascontiguousarray(kappa, dtype=np.float64)
    return lib().or_kappa_at(_p(kappa), ctypes.c_int(len(kappa)), ctypes.c_double(ds), ctypes.c_double(s))


def trajectory(model, cost, track, x0, V, eps=None):
    """(states [T+1][6], barrier values [T+1][1+n_obs]) of one control sequence."""
    V = np.ascontiguousarray(V, dtype=np.float64).reshape(-1, 2)
    T = V.shape[0]
    ta = _TrackArgs(track)
    xs = np.zeros((T + 1, 6))
    hs = np.zeros((T + 1, 1 + len(ta.obs)))
    mp, cp = model_array(model), cost_array(cost)
    lib().or_trajectory(_p(mp), _p(cp), *ta.args(), _p(x0), _p(V), ctypes.c_int(T),
                        _p(eps) if eps is not None else None, _p(xs), _p(hs))
    return xs, hs


def execute(model, x, u0, dist=None) -> np.ndarray:
    """Disturbed plant of eq. (26): x+ = f(x, u0) + w, with w acting on v_y and omega.
    The executed command is held inside the control box."""
    u0 = np.clip(np.asarray(u0, dtype=np.float64), model["u_lo"], model["u_hi"])
    xn = rk4(model, x, u0, model["dt"], 1)
    if dist is not None:
        xn[4] += dist[0]
        xn[5] += dist[1]
    return xn


def shift(V_plus) -> np.ndarray:
    """Warm start: drop the executed step, repeat the last one."""
    V_plus = np.asarray(V_plus).reshape(-1, 2)
    return np.concatenate([V_plus[1:], V_plus[-1:]], axis=0)
