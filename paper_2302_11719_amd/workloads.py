"""Seeded synthetic workloads for the Shield-MPPI sampled-rollout step.

This module produces INPUT DATA only: model and cost constants, track
geometry (circle or closed polyline sampled from a periodic cubic spline),
circular obstacles, initial states, ragged batch shapes and plant
disturbances.  It contains none of the method's arithmetic (no dynamics, no
cost, no sampling noise, no weighting) and it is the only module that both the
GPU path's callers and the FP64 oracle's callers share.

The paper's own workloads (the AutoRally simulator, its track and its
calibrated eight-state vehicle) are not available; these racing-shaped inputs
stand in for them.  Geometry is generated in FP64 with numpy's PCG64 streams
(seeded per purpose) and scipy's periodic cubic spline.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Six-state single-track vehicle: mass and wheelbase as stated for the
# workload; axle split, inertia, tyre stiffness and drive/drag constants
# chosen so that an explicit RK4 step of 0.05 s stays well inside its
# stability region (fastest lateral mode (Cf+Cr)/(m v_min) = 20 1/s).
MODEL = dict(m=3.0, lf=0.13, lr=0.13, Iz=3.0 * 0.13 * 0.13, Cf=30.0, Cr=30.0, a_max=4.0, c_v=0.5,
             v_min=1.0, dt=0.05, u_lo=(-0.4, -1.0), u_hi=(0.4, 1.0))

# Running cost on speed error and lateral deviation with a collision
# indicator, control-cost weight equal to lambda, DCBF penalty weight C and
# decay rate gamma (alpha = 1 - gamma).
COST = dict(v_g=4.0, q_v=1.0, q_ey=10.0, C_obs=100.0, phi_w=1.0, lambda_u=1.0, sigma=(0.2, 0.4),
            C_cbf=1.0e3, gamma=0.2)
LAMBDA = 1.0
WINDOW = 4

# Objectives for differentiation: the shield of Algorithm 1 (violation hinge
# only) and the "total cost plus squared violations" objective.
OBJ_SHIELD = dict(w_S=0.0, w_sq=0.0, w_lin=1.0, n_lin=1 << 30)
OBJ_TOTAL = dict(w_S=1.0, w_sq=1.0, w_lin=0.0, n_lin=0)

TRACK_SEED_BASE = 0x7AC0
OBST_SEED_BASE = 0x0B57
INIT_SEED_BASE = 0x1417
DIST_SEED_BASE = 0xD157
SHAPE_SEED = 0x5EA9
SEQ_SEED_BASE = 0x5E90


@dataclass
class Track:
    kind: int                       # 0 circle, 1 closed polyline
    circle: np.ndarray              # (3,) cx, cy, R  (zeros for a polyline)
    poly: np.ndarray                # (n, 5) ax, ay, dx, dy, 1/|d|^2  (empty for a circle)
    half_width: float
    obs: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))  # (n, 4) cx, cy, r_eff^2, r^2
    window: int = WINDOW


@dataclass
class Problem:
    K: int
    T: int
    track: Track
    x0: np.ndarray                  # (6,)
    V: np.ndarray                   # (T, 2) nominal control sequence
    pid: int = 0
    it: int = 0


def circle_track(R: float = 10.0, half_width: float = 1.0) -> Track:
    return Track(kind=0, circle=np.array([0.0, 0.0, R]), poly=np.zeros((0, 5)), half_width=half_width)


def polyline_from_vertices(P: np.ndarray) -> np.ndarray:
    """Closed polyline rows (ax, ay, dx, dy, 1/|d|^2) from vertices (n, 2)."""
    P = np.asarray(P, dtype=np.float64)
    D = np.roll(P, -1, axis=0) - P
    inv = 1.0 / np.einsum("ij,ij->i", D, D)
    return np.column_stack([P[:, 0], P[:, 1], D[:, 0], D[:, 1], inv])


def spline_control_points(seed: int, n_ctrl: int = 12, r0: float = 15.0, dr: float = 4.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(TRACK_SEED_BASE + seed))
    theta = 2.0 * math.pi * np.arange(n_ctrl) / n_ctrl
    r = r0 + dr * (2.0 * rng.random(n_ctrl) - 1.0)
    return np.column_stack([r * np.cos(theta), r * np.sin(theta)])


def spline_vertices(ctrl: np.ndarray, n_s: int = 512) -> np.ndarray:
    """Periodic C2 cubic spline through the control points (uniform knots), sampled
    at n_s parameter-uniform points (counter-clockwise)."""
    from scipy.interpolate import CubicSpline

    n = len(ctrl)
    knots = np.arange(n + 1, dtype=np.float64)
    pts = np.vstack([ctrl, ctrl[:1]])
    cs = CubicSpline(knots, pts, bc_type="periodic")
    s = n * np.arange(n_s, dtype=np.float64) / n_s
    return cs(s)


def spline_track(seed: int, half_width: float = 0.9, n_s: int = 512) -> Track:
    P = spline_vertices(spline_control_points(seed), n_s)
    return Track(kind=1, circle=np.zeros(3), poly=polyline_from_vertices(P), half_width=half_width)


def curvature_table(track: Track, n: int = 1024):
    """(kappa [n], ds): the centre line's signed curvature (left turns positive) on a
    uniform arclength grid s_k = k ds of the closed polyline, ds = length / n.  Vertex
    curvature = turning angle / mean adjacent segment length, then periodic linear
    interpolation in arclength.  A circle gives the constant 1/R."""
    if track.kind == 0:
        R = float(track.circle[2])
        return np.full(n, 1.0 / R), 2.0 * math.pi * R / n
    poly = track.poly
    seg = np.hypot(poly[:, 2], poly[:, 3])
    th = np.arctan2(poly[:, 3], poly[:, 2])
    dth = np.angle(np.exp(1j * (th - np.roll(th, 1))))
    kv = dth / (0.5 * (seg + np.roll(seg, 1)))
    sv = np.concatenate([[0.0], np.cumsum(seg)[:-1]])
    L = float(seg.sum())
    ds = L / n
    sk = np.arange(n) * ds
    kappa = np.interp(sk, np.concatenate([sv, [L]]), np.concatenate([kv, [kv[0]]]))
    return kappa, ds


# Wheels of the eight-state curvilinear model (the paper's state with front and
# rear wheel speeds): wheel radius, wheel inertia per axle, longitudinal slip
# stiffness per axle.  Chosen so that the wheel-spin modes (about
# C_x (1/m + r_w^2/I_w) / v_min = 35 1/s at the slowest) stay inside RK4's
# stability region at dt = 0.05 s.
WHEELS = dict(r_w=0.05, I_w=0.01, C_x=60.0)


def start_state_c8(vx: float = 3.0, e_y: float = 0.0, e_psi: float = 0.0, s: float = 0.0) -> np.ndarray:
    """Eight-state curvilinear start (v_x, v_y, r, omega_F, omega_R, e_psi, e_y, s): straight
    running with both wheels rolling freely (omega = v_x / r_w)."""
    w = vx / WHEELS["r_w"]
    return np.array([vx, 0.0, 0.0, w, w, e_psi, e_y, s])


def obstacles(track: Track, seed: int, n: int = 64, margin: float = 0.15, keep_clear: float = 5.0) -> np.ndarray:
    """Circular obstacles at seeded arclength positions and lateral offsets inside the
    track; radius U[0.2, 0.6]; rows (cx, cy, (r + margin)^2, r^2).  The first
    `keep_clear` metres after vertex 0 stay free so that the start state is safe."""
    rng = np.random.Generator(np.random.PCG64(OBST_SEED_BASE + seed))
    poly = track.poly
    seg_len = np.hypot(poly[:, 2], poly[:, 3])
    cum = np.concatenate([[0.0], np.cumsum(seg_len)])
    L = cum[-1]
    out = np.zeros((n, 4))
    for i in range(n):
        s = keep_clear + rng.random() * (L - keep_clear)
        lat = (2.0 * rng.random() - 1.0) * track.half_width
        r = 0.2 + 0.4 * rng.random()
        j = min(int(np.searchsorted(cum, s, side="right")) - 1, len(poly) - 1)
        f = (s - cum[j]) / seg_len[j]
        ax, ay, dx, dy = poly[j, :4]
        nx, ny = -dy / seg_len[j], dx / seg_len[j]
        out[i] = (ax + f * dx + lat * nx, ay + f * dy + lat * ny, (r + margin) ** 2, r * r)
    return out


def start_state(track: Track, vertex: int = 0, vx: float = 3.0) -> np.ndarray:
    if track.kind == 0:
        cx, cy, R = track.circle
        return np.array([cx + R, cy, math.pi / 2.0, vx, 0.0, 0.0])
    ax, ay, dx, dy = track.poly[vertex, :4]
    return np.array([ax, ay, math.atan2(dy, dx), vx, 0.0, 0.0])


def config0() -> Problem:
    """Single iteration, circle R=10 m, half width 1 m, K=256, T=20, FP64."""
    tr = circle_track(10.0, 1.0)
    return Problem(K=256, T=20, track=tr, x0=start_state(tr), V=np.zeros((20, 2)), pid=0, it=0)


def config1(K: int = 4096, T: int = 50, seed: int = 0) -> Problem:
    """Closed loop on a seeded spline track, half width 0.9 m, K=4096, T=50."""
    tr = spline_track(seed, 0.9)
    return Problem(K=K, T=T, track=tr, x0=start_state(tr), V=np.zeros((T, 2)), pid=seed, it=0)


def config2_shapes(B: int = 512, k_lo: int = 256, k_hi: int = 16384, t_lo: int = 20, t_hi: int = 100):
    rng = np.random.Generator(np.random.PCG64(SHAPE_SEED))
    K = np.rint(np.exp(rng.uniform(math.log(k_lo), math.log(k_hi), size=B))).astype(np.int64)
    T = rng.integers(t_lo, t_hi + 1, size=B).astype(np.int64)
    return K, T


def config2(B: int = 512, k_lo: int = 256, k_hi: int = 16384, t_lo: int = 20, t_hi: int = 100):
    """Ragged batch: own spline track and random start per problem."""
    Ks, Ts = config2_shapes(B, k_lo, k_hi, t_lo, t_hi)
    out = []
    for b in range(B):
        tr = spline_track(b, 0.9)
        rng = np.random.Generator(np.random.PCG64(INIT_SEED_BASE + b))
        vert = int(rng.integers(0, len(tr.poly)))
        vx = float(rng.uniform(1.0, 5.0))
        out.append(Problem(K=int(Ks[b]), T=int(Ts[b]), track=tr, x0=start_state(tr, vert, vx),
                           V=np.zeros((int(Ts[b]), 2)), pid=b, it=0))
    return out


def config3(B: int = 64, K: int = 2048, T: int = 50):
    """Differentiation workload: 64 problems, K=2048, T=50 on their own tracks."""
    out = []
    for b in range(B):
        tr = spline_track(b, 0.9)
        out.append(Problem(K=K, T=T, track=tr, x0=start_state(tr), V=np.zeros((T, 2)), pid=b, it=0))
    return out


def config4(K: int = 65536, T: int = 100, n_obs: int = 64, seed: int = 0) -> Problem:
    """One large problem with 64 circular obstacles on the track."""
    tr = spline_track(seed, 0.9)
    tr.obs = obstacles(tr, seed, n_obs)
    return Problem(K=K, T=T, track=tr, x0=start_state(tr), V=np.zeros((T, 2)), pid=seed, it=0)


def identical_batch(B: int, K: int = 4096, T: int = 50):
    """B copies of the K=4096, T=50 problem shape, each on its own seeded track."""
    out = []
    for b in range(B):
        tr = spline_track(b, 0.9)
        out.append(Problem(K=K, T=T, track=tr, x0=start_state(tr), V=np.zeros((T, 2)), pid=b, it=0))
    return out


def disturbances(seed: int, steps: int, sigma: float = 0.3) -> np.ndarray:
    """Plant disturbance (steps, 2) on (v_y, omega), eq. (26)."""
    rng = np.random.Generator(np.random.PCG64(DIST_SEED_BASE + seed))
    return sigma * rng.standard_normal((steps, 2))


def test_sequences(n: int, T: int, seed: int = 0, scale: float = 0.5) -> np.ndarray:
    """Seeded control sequences (n, T, 2) strictly inside the control box."""
    rng = np.random.Generator(np.random.PCG64(SEQ_SEED_BASE + seed))
    lo = np.array(MODEL["u_lo"])
    hi = np.array(MODEL["u_hi"])
    return (lo + (hi - lo) * (0.5 + scale * (rng.random((n, T, 2)) - 0.5)))


def round_to_f32(p: Problem) -> Problem:
    """Same problem with every float input rounded to FP32 (so that an FP32 device run
    and the FP64 oracle see identical geometry, start state and controls)."""
    f = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    tr = p.track
    tr2 = Track(kind=tr.kind, circle=f(tr.circle), poly=f(tr.poly), half_width=float(np.float32(tr.half_width)),
                obs=f(tr.obs), window=tr.window)
    return Problem(K=p.K, T=p.T, track=tr2, x0=f(p.x0), V=f(p.V), pid=p.pid, it=p.it)


def params_f32(model: dict, cost: dict):
    """Model/cost constants rounded to FP32 (matching what an FP32 device run uses)."""
    r = lambda v: float(np.float32(v))
    m2 = {k: (tuple(r(x) for x in v) if isinstance(v, tuple) else r(v)) for k, v in model.items()}
    c2 = {k: (tuple(r(x) for x in v) if isinstance(v, tuple) else r(v)) for k, v in cost.items()}
    return m2, c2


def wheels_f32(wheels: dict = None) -> dict:
    return {k: float(np.float32(v)) for k, v in (wheels or WHEELS).items()}
