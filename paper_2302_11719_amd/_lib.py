"""ctypes binding of libsmppi (the C ABI declared in include/smppi.h).

Argument marshalling only: every step of the sampled-rollout path runs in the
library's HIP kernels.  PyTorch supplies device memory (tensors' data
pointers) and the current stream.  Importing this module never falls back to
any other implementation: if the shared library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsmppi.so")

c_i32, c_u32, c_i64, c_f64, c_vp = ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p

F32, F64 = 0, 1
STATUS = {0: "ok", 1: "invalid argument", 2: "shape", 3: "dtype", 4: "no device", 5: "hip error",
          6: "unsupported", 7: "non-finite"}
ERR_NO_DEVICE = 4

# Symbols declared in include/smppi.h (checked by the CPU test suite).
ABI_VERSION = 7  # SMPPI_ABI_VERSION of include/smppi.h this binding matches
EXPORTS = ("smppi_rollout_curvilinear", "smppi_rollout_backward_curvilinear", "smppi_shield_repair_curvilinear",
           "smppi_execute_curvilinear", "smppi_create", "smppi_destroy", "smppi_last_error", "smppi_status_string", "smppi_abi_version",
           "smppi_reserve_batch", "smppi_device_errors", "smppi_rollout", "smppi_weights", "smppi_update",
           "smppi_rollout_backward", "smppi_rollout_backward_noalloc", "smppi_shield_repair", "smppi_execute", "smppi_plan_create",
           "smppi_plan_launch", "smppi_plan_destroy", "smppi_plan_info", "smppi_plan_launch_profiled",
           "smppi_plan_stage_ms", "smppi_plan_kernel_ms", "smppi_autotune", "smppi_autotune_candidates",
           "smppi_autotune_key", "smppi_debug_philox")


class Model(ctypes.Structure):
    _fields_ = [("m", c_f64), ("lf", c_f64), ("lr", c_f64), ("Iz", c_f64), ("Cf", c_f64), ("Cr", c_f64),
                ("a_max", c_f64), ("c_v", c_f64), ("v_min", c_f64), ("dt", c_f64), ("u_lo", c_f64 * 2),
                ("u_hi", c_f64 * 2)]


class Cost(ctypes.Structure):
    _fields_ = [("v_g", c_f64), ("q_v", c_f64), ("q_ey", c_f64), ("C_obs", c_f64), ("phi_w", c_f64),
                ("lambda_u", c_f64), ("sigma", c_f64 * 2), ("C_cbf", c_f64), ("gamma", c_f64)]


class Noise(ctypes.Structure):
    _fields_ = [("seed", c_u32), ("nominal", c_i32)]


class Batch(ctypes.Structure):
    _fields_ = [("n_problems", c_i32), ("k_max", c_i32), ("t_max", c_i32), ("pid_base", c_i32), ("dtype", c_i32),
                ("k_off", c_vp), ("t_off", c_vp)]


class Track(ctypes.Structure):
    _fields_ = [("poly_off", c_vp), ("poly", c_vp), ("circle", c_vp), ("half_width", c_vp), ("obs_off", c_vp),
                ("obs", c_vp), ("window", c_i32), ("poly_max", c_i32), ("obs_max", c_i32)]


class CurvTrack(ctypes.Structure):
    _fields_ = [("kappa_off", c_vp), ("kappa", c_vp), ("ds", c_vp), ("half_width", c_vp), ("n_max", c_i32)]


class Wheels(ctypes.Structure):
    _fields_ = [("r_w", c_f64), ("I_w", c_f64), ("C_x", c_f64)]


class Objective(ctypes.Structure):
    _fields_ = [("w_S", c_f64), ("w_sq", c_f64), ("w_lin", c_f64), ("n_lin", c_i32)]


class RepairOpts(ctypes.Structure):
    _fields_ = [("n_steps", c_i32), ("step", c_f64), ("objective", Objective), ("method", c_i32),
                ("memory", c_i32)]


REPAIR_METHODS = {"gradient": 0, "lbfgs": 1}


def repair_opts(n_steps: int, step: float, objective: dict, method: str = "gradient", memory: int = 5) -> RepairOpts:
    """smppi_repair_opts from Python values (method "gradient" = Algorithm 1, "lbfgs")."""
    return RepairOpts(int(n_steps), float(step), objective_struct(objective), REPAIR_METHODS[method],
                      int(memory) if method == "lbfgs" else 0)


class PlanOpts(ctypes.Structure):
    _fields_ = [("lambda_", c_f64), ("repair", c_i32), ("repair_opts", RepairOpts), ("execute", c_i32),
                ("dist", c_vp), ("n_dist", c_i32), ("block", c_i32), ("tile", c_i32), ("grid", c_i32),
                ("use_graph", c_i32), ("pipeline", c_i32), ("fuse_shield", c_i32)]


class PlanBuffers(ctypes.Structure):
    _fields_ = [("x0", c_vp), ("V", c_vp), ("iter", c_vp), ("S", c_vp), ("V_plus", c_vp), ("stats", c_vp),
                ("V_safe", c_vp)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("pipeline", c_i32), ("block", c_i32), ("tile", c_i32), ("grid", c_i32),
                ("kernel_ms", ctypes.c_float)]


P = ctypes.POINTER

_SIGS = {
    "smppi_create": (c_i32, [ctypes.c_int, P(c_vp)]),
    "smppi_destroy": (None, [c_vp]),
    "smppi_last_error": (ctypes.c_char_p, [c_vp]),
    "smppi_status_string": (ctypes.c_char_p, [c_i32]),
    "smppi_abi_version": (ctypes.c_int, []),
    "smppi_reserve_batch": (c_i32, [c_vp, P(Batch)]),
    "smppi_device_errors": (c_i32, [c_vp, P(c_u32)]),
    "smppi_rollout_curvilinear": (c_i32, [c_vp, P(Batch), P(Model), P(Wheels), P(Cost), P(Noise), P(CurvTrack),
                                          c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "smppi_rollout_backward_curvilinear": (c_i32, [c_vp, P(Batch), P(Model), P(Wheels), P(Cost), P(Noise),
                                                   P(CurvTrack), c_vp, c_vp, c_vp, c_vp, P(Objective), c_vp, c_vp]),
    "smppi_shield_repair_curvilinear": (c_i32, [c_vp, P(Batch), P(Model), P(Wheels), P(Cost), P(CurvTrack), c_vp,
                                                c_vp, P(RepairOpts), c_vp, c_vp]),
    "smppi_execute_curvilinear": (c_i32, [c_vp, P(Batch), P(Model), P(Wheels), P(CurvTrack), c_vp, c_vp, c_vp,
                                          c_i32, c_vp, c_vp, c_vp, c_vp]),
    "smppi_rollout": (c_i32, [c_vp, P(Batch), P(Model), P(Cost), P(Noise), P(Track), c_vp, c_vp, c_vp, c_vp, c_vp,
                              c_vp]),
    "smppi_weights": (c_i32, [c_vp, P(Batch), c_vp, c_f64, c_vp, c_vp, c_vp]),
    "smppi_update": (c_i32, [c_vp, P(Batch), P(Model), P(Cost), P(Noise), c_vp, c_vp, c_vp, c_vp, c_vp]),
    "smppi_rollout_backward": (c_i32, [c_vp, P(Batch), P(Model), P(Cost), P(Noise), P(Track), c_vp, c_vp, c_vp,
                                       c_vp, P(Objective), c_vp, c_vp]),
    "smppi_rollout_backward_noalloc": (c_i32, [c_vp, P(Batch), P(Model), P(Cost), P(Noise), P(Track), c_vp, c_vp,
                                               c_vp, c_vp, P(Objective), c_vp, c_vp]),
    "smppi_shield_repair": (c_i32, [c_vp, P(Batch), P(Model), P(Cost), P(Track), c_vp, c_vp, P(RepairOpts), c_vp,
                                    c_vp]),
    "smppi_execute": (c_i32, [c_vp, P(Batch), P(Model), c_vp, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp]),
    "smppi_plan_create": (c_i32, [c_vp, P(Batch), P(Model), P(Cost), P(Noise), P(Track), P(PlanOpts),
                                  P(PlanBuffers), P(c_vp)]),
    "smppi_plan_launch": (c_i32, [c_vp, c_vp]),
    "smppi_plan_destroy": (None, [c_vp]),
    "smppi_plan_info": (c_i32, [c_vp, P(c_i32), P(c_i32), P(c_i32), P(c_i32)]),
    "smppi_plan_launch_profiled": (c_i32, [c_vp, c_vp]),
    "smppi_plan_stage_ms": (c_i32, [c_vp, P(ctypes.c_float), P(ctypes.c_float), P(ctypes.c_float)]),
    "smppi_plan_kernel_ms": (c_i32, [c_vp, P(ctypes.c_float), P(ctypes.c_float)]),
    "smppi_autotune": (c_i32, [c_vp, P(Batch), P(Model), P(Cost), P(Noise), P(Track), c_f64, P(PlanBuffers),
                               P(TuneEntry), c_i32, c_i32, c_i32, ctypes.c_char_p, c_i32, P(TuneEntry), P(c_i32),
                               P(TuneEntry), c_i32, P(c_i32), c_vp]),
    "smppi_autotune_candidates": (c_i32, [c_i32, P(TuneEntry), c_i32]),
    "smppi_autotune_key": (c_i32, [c_i32, P(c_i64), P(c_i32), c_i32, c_i32, ctypes.c_char_p, c_i32]),
    "smppi_debug_philox": (c_i32, [c_vp, c_vp, P(c_u32), c_i64, c_vp, c_vp]),
}

_lock = threading.Lock()
_lib = None


class SmppiError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"smppi: {STATUS.get(status, status)}: {msg}")


def lib():
    """Load libsmppi.so (built by __graft_entry__.build()); raises if it is missing."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                                  "(python paper_2302_11719_amd/build.py)")
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            if L.smppi_abi_version() != ABI_VERSION:
                raise ImportError(f"libsmppi ABI version {L.smppi_abi_version()}, binding expects {ABI_VERSION}: "
                                  "rebuild the library")
            _lib = L
    return _lib


def model_struct(d: dict) -> Model:
    m = Model()
    for k in ("m", "lf", "lr", "Iz", "Cf", "Cr", "a_max", "c_v", "v_min", "dt"):
        setattr(m, k, float(d[k]))
    m.u_lo[0], m.u_lo[1] = d["u_lo"]
    m.u_hi[0], m.u_hi[1] = d["u_hi"]
    return m


def cost_struct(d: dict) -> Cost:
    c = Cost()
    for k in ("v_g", "q_v", "q_ey", "C_obs", "phi_w", "lambda_u", "C_cbf", "gamma"):
        setattr(c, k, float(d[k]))
    c.sigma[0], c.sigma[1] = d["sigma"]
    return c


def wheels_struct(d: dict) -> Wheels:
    return Wheels(float(d["r_w"]), float(d["I_w"]), float(d["C_x"]))


def objective_struct(d: dict) -> Objective:
    return Objective(float(d["w_S"]), float(d["w_sq"]), float(d["w_lin"]), int(min(d["n_lin"], 2 ** 31 - 1)))
