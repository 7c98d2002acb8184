"""Benchmark of the Shield-MPPI sampled-rollout step on one MI355X.

Headline workload: the closed-loop configuration, K = 4096 samples, T = 50 steps,
one problem on a seeded spline track (12 control points, radius 15 +- 4 m,
half width 0.9 m), disturbance sigma = 0.3 on v_y and omega.  One timed step is
one receding-horizon Shield-MPPI iteration run by the batched plan as one
kernel launch: fused rollout + softmax weights + update, then the shield (10
projected gradient steps of the hand-written adjoint, step 0.05) and execute +
warm start in the workgroup that combined the problem.  value = rollout-steps/s = K*T*steps / elapsed.

Also measured in the same run (reported beside the headline): the plain
per-call form (rollout, weights, update, execute launches, no shield), the
batched plan on B identical-shape problems vs the plain per-problem loop, the
512-problem ragged batch, the K=65536/T=100/64-obstacle rollout, the stage
split (the headline with the shield as a kernel of its own), the dominant
kernel's roofline, and the FP64 CPU oracle on a bounded sample of the headline
workload.

usage: python bench.py [--gpus 1] [--steps 500] [--warmup 20] [--skip-cpu] [--quick]
                       [--forms split,active,plain,identical,ragged,large,c0,c3,c4adj,shield,autotune,sweep,
                                curvilinear]
                       [--copy-calibration-mib N]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic FP32 operation counts per rollout-step (FMA = 2, transcendental = 1,
# compares/selects not counted), counted term by term from the device code.
FLOP_STEP_POLY = 345      # noise, clip, cost, RK4 (4 derivative evaluations), 9-segment window, DCBF
FLOP_STEP_PER_OBS = 9     # one circular obstacle barrier + penalty + indicator test
FLOP_UPDATE_STEP = 4      # w * eps' accumulated for two controls
FLOP_STEP_C8 = 400        # eight-state curvilinear model: 4 derivative evaluations of ~69 (tyre and wheel forces,
                          # curvature lookup, Frenet kinematics), RK4 stages and combine 96, noise, clip, cost, DCBF
PEAK_FP32 = 157.3e12      # MI355X FP32 vector peak (packed FMA on every lane)
PEAK_HBM = 8.0e12
FORMS = ("split", "active", "plain", "identical", "ragged", "large", "c0", "c3", "c4adj", "shield", "autotune", "sweep",
         "curvilinear")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_fused_K4096_T50_hbm_traffic.md")
# The paper's own control rates (Sec. VI-G, the vehicle experiment and its results table):
# context only, other vehicle model, horizon, precision and hardware.
PAPER_RATES = [
    {"controller": "MPPI(a)", "samples": 10000, "rate_hz": 150, "hardware": "NVIDIA GTX 1080 Ti"},
    {"controller": "Shield-MPPI(a)", "samples": 10000, "rate_hz": 55, "hardware": "NVIDIA GTX 1080 Ti"},
    {"controller": "MPPI(b)", "samples": 20, "rate_hz": 235, "hardware": "Intel Skylake quad-core i7"},
    {"controller": "Shield-MPPI(b)", "samples": 20, "rate_hz": 220, "hardware": "Intel Skylake quad-core i7"},
]


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline only (same as --forms none)")
    ap.add_argument("--forms", default="all",
                    help="comma list of the extra forms to run: split (the headline with the shield as a "
                         "kernel of its own), active (the headline from a start where the shield fires), plain, "
                         "identical, ragged, large, c0 (FP64), c3 (adjoint repair), c4adj (free-energy "
                         "adjoint), shield, autotune, sweep, curvilinear (or all/none); without split and "
                         "active, every k_fused launch of the run is the headline kernel")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (scale for HBM byte counters)")
    args = ap.parse_args()
    forms = set() if args.quick or args.forms == "none" else (
        set(FORMS) if args.forms == "all" else set(args.forms.split(",")))
    if forms - set(FORMS):
        ap.error(f"unknown forms {sorted(forms - set(FORMS))}")
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch

    from paper_2302_11719_amd import core
    from paper_2302_11719_amd import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)
    ctx = core.Context(0)
    M, C = W.params_f32(W.MODEL, W.COST)
    lam = W.LAMBDA
    rep = dict(n_steps=10, step=0.05, objective=W.OBJ_SHIELD)
    K, T = 4096, 50
    steps, warm = args.steps, args.warmup
    seed = 0

    def sync():
        torch.cuda.synchronize()

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        sync()
        dst.copy_(src)
        sync()
        _log(f"copy calibration: {n} bytes read + {n} bytes written")
        del src, dst

    # ------------------------------------------------------------------ headline
    prob = W.round_to_f32(W.config1(K=K, T=T))
    n_dist = warm + 2 * steps + 8
    dist = torch.as_tensor(W.disturbances(0, n_dist).astype(np.float32).reshape(n_dist, 1, 2), device="cuda")
    db = core.DeviceBatch([prob], dtype=torch.float32)
    plan = core.Plan(ctx, db, M, C, seed, lam, repair=rep, execute=True, dist=dist, use_graph=True)
    _log(f"headline: K={K} T={T} plan={plan.info()} warmup={warm} steps={steps}")
    for _ in range(warm):
        plan.launch()
    sync()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        plan.launch()
    ev1.record()
    sync()
    wall = time.perf_counter() - t0
    assert ctx.device_errors() == 0
    ms_per_step = 1e3 * wall / steps
    value = K * T * steps / wall
    # per-iteration distribution, measured after the timed region (an event between
    # launches costs a few microseconds of its own)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    evs[0].record()
    for i in range(steps):
        plan.launch()
        evs[i + 1].record()
    sync()
    per_iter = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(steps)])
    _log(f"  {ms_per_step:.4f} ms/iter (events {ev0.elapsed_time(ev1) / steps:.4f}; with an event per iteration: "
         f"mean {per_iter.mean():.4f}, median {np.median(per_iter):.4f}), {value:.4g} rollout-steps/s")

    # The headline launch is one kernel (fused rollout/weights/update, shield, plant):
    # its duration from kernel-stamped events on an eager copy of the same plan.
    n_prof = min(steps, 100)
    db_f = core.DeviceBatch([prob], dtype=torch.float32)
    plan_f = core.Plan(ctx, db_f, M, C, seed, lam, repair=rep, execute=True, dist=dist, use_graph=False)
    kl = []
    for i in range(warm + n_prof):
        plan_f.launch_profiled()
        if i >= warm:
            kl.append(plan_f.kernel_ms()[0])
    plan_f.close()
    stage = dict(launch_kernel_ms=float(np.mean(kl)))
    if "split" in forms:
        stage.update(stage_split(ctx, prob, M, C, seed, lam, rep, dist, warm, n_prof))
    _log(f"  stages: {stage}")

    # roofline of the one kernel: the rollouts and update (the shield's nominal pass,
    # T steps of one trajectory, is not counted)
    dominant = "k_fused"
    flops = K * T * (FLOP_STEP_POLY + FLOP_UPDATE_STEP)
    dur = stage["launch_kernel_ms"] * 1e-3
    achieved = flops / dur
    from paper_2302_11719_amd.profile_summary import load_traffic

    traffic, why = load_traffic(TRAFFIC_SUMMARY, dominant)
    roofline = {"bound": "alu", "kernel": "k_fused (rollout, weights, update, shield, plant step)",
                "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32,
                "traffic": traffic, "traffic_unit": "bytes/launch", "flop_per_launch": flops,
                "avg_launch_ms": dur * 1e3}
    if traffic is None:
        roofline["traffic_note"] = why

    result = {
        "metric": "rollout-steps/s and ms/MPPI iter (K=4096,T=50); batched+adjoint vs plain",
        "value": value, "unit": "rollout-steps/s", "n_gpus": 1, "steps": steps, "warmup": warm,
        "ms_per_step": ms_per_step, "ms_per_step_median_evented": float(np.median(per_iter)),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "closed-loop Shield-MPPI iteration (batched+adjoint plan, one launch): "
                               "K=4096, T=50, 1 problem, spline track, shield 10x0.05, plant disturbance 0.3",
                   "K": K, "T": T, "problems": 1, "repair_steps": 10, "parallelism": "single-gpu"},
        "stages_ms": stage,
        "roofline": roofline,
        "paper_context": {"note": "the paper's reported control rates on its vehicle's hardware (context only; "
                                  "other model, horizon and hardware)", "rates": PAPER_RATES,
                          "this_run_rate_hz": 1e3 / ms_per_step, "this_run_samples": K},
    }

    if forms:
        result["forms"] = extra_forms(ctx, core, W, M, C, lam, rep, K, T, sync, forms)
    if not args.skip_cpu:
        result["cpu_baseline"] = cpu_baseline(W, K, T, lam, rep)
    print(json.dumps(result), flush=True)



def stage_split(ctx, prob, M, C, seed, lam, rep, dist, warm, n_prof):
    """Stage split of the headline work with the shield as a kernel of its own
    (kernel-stamped events on the fused and shield kernels)."""
    import torch

    from paper_2302_11719_amd import core

    db_p = core.DeviceBatch([prob], dtype=torch.float32)
    plan_p = core.Plan(ctx, db_p, M, C, seed, lam, repair=rep, execute=True, dist=dist, use_graph=False,
                       fuse_shield=-1)
    fused, repair_t, active, kf, kr = [], [], [], [], []
    for i in range(warm + n_prof):
        plan_p.launch_profiled()
        f, r, _ = plan_p.stage_ms()
        k1, k2 = plan_p.kernel_ms()
        if i >= warm:
            fused.append(f)
            repair_t.append(r)
            kf.append(k1)
            kr.append(k2)
            # the shield changed the MPPI output (some DCBF condition was violated)
            active.append(not torch.equal(plan_p.V_safe, plan_p.V_plus))
    plan_p.close()
    act = np.array(active)
    kr = np.array(kr)
    return dict(split_rollout_weights_update_kernel_ms=float(np.mean(kf)),
                split_shield_plant_kernel_ms=float(kr.mean()), shield_active_fraction=float(act.mean()),
                shield_kernel_ms_when_active=float(kr[act].mean()) if act.any() else None,
                shield_kernel_ms_when_idle=float(kr[~act].mean()) if (~act).any() else None)

def _capture(fn):
    """fn's launches captured into a torch CUDA graph (the library's calls allocate and
    synchronise nothing, so only their kernels are recorded)."""
    import torch

    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


def _time(fn, n, warm, sync):
    for _ in range(warm):
        fn()
    sync()
    t0 = time.perf_counter()
    for _ in range(n):
        fn()
    sync()
    return (time.perf_counter() - t0) / n


def extra_forms(ctx, core, W, M, C, lam, rep, K, T, sync, forms):
    out = {}
    seed = 0
    if "active" in forms:
        _form_active(ctx, core, W, M, C, lam, rep, K, T, sync, out, seed)
    if "plain" in forms:
        _form_plain(ctx, core, W, M, C, lam, K, T, sync, out, seed)
    if "identical" in forms:
        _form_identical(ctx, core, W, M, C, lam, rep, K, T, sync, out, seed)
    if "ragged" in forms:
        _form_ragged(ctx, core, W, M, C, lam, sync, out, seed)
    if "large" in forms:
        _form_large(ctx, core, W, M, C, lam, sync, out, seed)
    if "c0" in forms:
        _form_c0(ctx, core, W, lam, sync, out, seed)
    if "c3" in forms:
        _form_c3(ctx, core, W, M, C, lam, rep, sync, out, seed)
    if "c4adj" in forms:
        _form_c4_adjoint(ctx, core, W, M, C, lam, sync, out, seed)
    if "shield" in forms:
        _form_shield(ctx, core, W, M, C, rep, sync, out)
    if "autotune" in forms:
        _form_autotune(ctx, core, W, M, C, lam, sync, out, seed)
    if "sweep" in forms:
        _form_sweep(ctx, out)
    if "curvilinear" in forms:
        _form_curvilinear(ctx, core, W, M, C, sync, out, seed)
    return out


def _active_fraction(db, V_plus, V_safe):
    """Fraction of problems whose shield output differs from the MPPI output (the shield
    changed the controls because some DCBF condition was violated)."""
    a, b = db.controls(V_plus), db.controls(V_safe)
    return float(np.mean([not np.array_equal(x, y) for x, y in zip(a, b)]))


def _offset_start(W, tr, lat, dpsi, vx):
    x0 = W.start_state(tr, vx=vx)
    ax, ay, dx, dy = tr.poly[0, :4]
    n = float(np.hypot(dx, dy))
    x0[0] += lat * (-dy / n)
    x0[1] += lat * (dx / n)
    x0[2] += dpsi
    return x0


def _form_active(ctx, core, W, M, C, lam, rep, K, T, sync, out, seed):
    """The headline launch (K = 4096, T = 50, shield 10 x 0.05) from a start 0.5 m off the
    centre line, heading 0.5 rad towards the edge at 5 m/s: the MPPI output violates the
    DCBF condition and the shield repairs it in every launch (no plant step, so every
    launch repeats the same iteration).  Beside it: the same launch from the headline's
    start (shield idle)."""
    import torch

    res = {}
    for name, off in (("active", (0.5, 0.5, 5.0)), ("idle", None)):
        p = W.config1(K=K, T=T)
        if off:
            p.x0 = _offset_start(W, p.track, *off)
        p = W.round_to_f32(p)
        db = core.DeviceBatch([p], dtype=torch.float32)
        pl = core.Plan(ctx, db, M, C, seed, lam, repair=rep, execute=False, use_graph=True)
        dt = _time(pl.launch, 200, 20, sync)
        frac = _active_fraction(db, pl.V_plus, pl.V_safe)
        pl.close()
        plp = core.Plan(ctx, db, M, C, seed, lam, repair=rep, execute=False, use_graph=False)
        kl = []
        for i in range(120):
            plp.launch_profiled()
            if i >= 20:
                kl.append(plp.kernel_ms()[0])
        plp.close()
        res[name] = {"ms_per_iter": dt * 1e3, "rollout_steps_per_s": K * T / dt, "kernel_ms": float(np.mean(kl)),
                     "shield_active_fraction": frac}
    out["headline_shield_active_vs_idle"] = res
    _log(f"  shield active vs idle: {res}")


def _form_plain(ctx, core, W, M, C, lam, K, T, sync, out, seed):
    import torch

    # plain per-call form on the headline problem: rollout, weights, update, execute (no shield)
    prob = W.round_to_f32(W.config1(K=K, T=T))
    db = core.DeviceBatch([prob], dtype=torch.float32)

    def plain_iter():
        S = core.rollout(ctx, db, M, C, seed)
        w, _ = core.weights(ctx, db, S, lam)
        Vp = core.update(ctx, db, M, C, seed, w)
        core.execute(ctx, db, M, Vp, Vp)

    dt = _time(plain_iter, 200, 20, sync)
    out["plain_single"] = {"ms_per_iter": dt * 1e3, "rollout_steps_per_s": K * T / dt, "shield": False}
    # the same four calls captured once in a HIP graph (torch's graph API) and replayed
    g = _capture(plain_iter)
    dt = _time(g.replay, 200, 20, sync)
    out["plain_single"]["graph_ms_per_iter"] = dt * 1e3
    del g

    # batched plan without the shield on the same problem (isolates fusion + graph)
    db2 = core.DeviceBatch([prob], dtype=torch.float32)
    pl = core.Plan(ctx, db2, M, C, seed, lam, execute=True, use_graph=True)
    dt = _time(pl.launch, 200, 20, sync)
    out["batched_single_noshield"] = {"ms_per_iter": dt * 1e3, "rollout_steps_per_s": K * T / dt}
    pl.close()
    _log(f"  plain single {out['plain_single']}, batched no-shield {out['batched_single_noshield']}")


def _form_identical(ctx, core, W, M, C, lam, rep, K, T, sync, out, seed):
    import torch

    # B identical-shape problems: plain per-problem loop vs the batched+adjoint plan
    for B in (8, 64, 512):
        probs = [W.round_to_f32(p) for p in W.identical_batch(B, K, T)]
        dbs = [core.DeviceBatch([p], dtype=torch.float32, pid_base=b) for b, p in enumerate(probs)]

        def loop():
            for d in dbs:
                S = core.rollout(ctx, d, M, C, seed)
                w, _ = core.weights(ctx, d, S, lam)
                core.update(ctx, d, M, C, seed, w)

        n_it = 3 if B == 512 else 10
        t_plain = _time(loop, n_it, 1, sync)
        dbB = core.DeviceBatch(probs, dtype=torch.float32)
        plB = core.Plan(ctx, dbB, M, C, seed, lam, repair=rep, use_graph=True)
        t_b = _time(plB.launch, 20, 3, sync)  # the batched launch is cheap: more repetitions
        out[f"identical_B{B}"] = {"plain_loop_ms": t_plain * 1e3, "batched_adjoint_ms": t_b * 1e3,
                                  "plain_rollout_steps_per_s": B * K * T / t_plain,
                                  "batched_rollout_steps_per_s": B * K * T / t_b, "speedup": t_plain / t_b,
                                  "shield_active_fraction": _active_fraction(dbB, plB.V_plus, plB.V_safe)}
        _log(f"  B={B}: {out[f'identical_B{B}']}")
        plB.close()
        del dbs, dbB


def _form_ragged(ctx, core, W, M, C, lam, sync, out, seed):
    import torch

    # the 512-problem ragged batch (K log-uniform [256, 16384], T uniform [20, 100])
    probs = [W.round_to_f32(p) for p in W.config2()]
    steps_total = sum(p.K * p.T for p in probs)
    dbR = core.DeviceBatch(probs, dtype=torch.float32)
    plR = core.Plan(ctx, dbR, M, C, seed, lam, use_graph=True)
    t_r = _time(plR.launch, 20, 3, sync)
    dbs = [core.DeviceBatch([p], dtype=torch.float32, pid_base=b) for b, p in enumerate(probs)]

    def loopR():
        for d in dbs:
            S = core.rollout(ctx, d, M, C, seed)
            w, _ = core.weights(ctx, d, S, lam)
            core.update(ctx, d, M, C, seed, w)

    t_rp = _time(loopR, 2, 1, sync)
    out["ragged_B512"] = {"rollout_steps": steps_total, "batched_ms": t_r * 1e3,
                          "batched_rollout_steps_per_s": steps_total / t_r, "plain_loop_ms": t_rp * 1e3,
                          "plain_rollout_steps_per_s": steps_total / t_rp, "plan": plR.info()}
    _log(f"  ragged: {out['ragged_B512']}")
    plR.close()
    del dbs


def _form_large(ctx, core, W, M, C, lam, sync, out, seed):
    import torch

    # large single problem: K=65536, T=100, 64 obstacles (rollout kernel alone and the plan)
    p4 = W.round_to_f32(W.config4())
    db4 = core.DeviceBatch([p4], dtype=torch.float32)
    S4 = db4.new_S()
    t4 = _time(lambda: core.rollout(ctx, db4, M, C, seed, S=S4), 20, 3, sync)
    fl4 = (FLOP_STEP_POLY + 64 * FLOP_STEP_PER_OBS) * p4.K * p4.T
    pl4 = core.Plan(ctx, db4, M, C, seed, lam, use_graph=True)
    t4p = _time(pl4.launch, 20, 3, sync)
    out["large_K65536_T100_obs64"] = {
        "rollout_ms": t4 * 1e3, "rollout_steps_per_s": p4.K * p4.T / t4,
        "rollout_achieved_TFLOPs": fl4 / t4 / 1e12, "rollout_frac_fp32_peak": fl4 / t4 / PEAK_FP32,
        "flop_note": "algorithmic: every obstacle barrier on every step; the kernel skips the obstacle terms "
                     "that are exactly zero for every sample of a wave, so it executes fewer (rocprofv3 counters)",
        "plan_ms": t4p * 1e3, "plan_rollout_steps_per_s": p4.K * p4.T / t4p}
    _log(f"  large: {out['large_K65536_T100_obs64']}")
    pl4.close()


def _form_c0(ctx, core, W, lam, sync, out, seed):
    """Config 0: one plain MPPI iteration in FP64 (K = 256, T = 20, circle track):
    rollout, weights, update as separate calls, and the same three captured once in a
    HIP graph; latency per iteration."""
    import torch

    p = W.config0()
    db = core.DeviceBatch([p], dtype=torch.float64)

    def it():
        S = core.rollout(ctx, db, W.MODEL, W.COST, seed)
        w, _ = core.weights(ctx, db, S, lam)
        core.update(ctx, db, W.MODEL, W.COST, seed, w)

    dt = _time(it, 500, 50, sync)
    g = _capture(it)
    dg = _time(g.replay, 500, 50, sync)
    del g
    out["c0_fp64_K256_T20"] = {"ms_per_iter": dt * 1e3, "rollout_steps_per_s": p.K * p.T / dt, "dtype": "f64",
                               "graph_ms_per_iter": dg * 1e3}
    _log(f"  c0: {out['c0_fp64_K256_T20']}")


def _form_c3(ctx, core, W, M, C, lam, rep, sync, out, seed):
    """Config 3: 64 problems x (K = 2048, T = 50); the shield's objective is the total cost
    plus the summed squared DCBF violations, whose gradient does not vanish, so all 10
    projected-gradient steps (0.05) run on every problem.  Batched+adjoint plan (one
    fused launch + the repair kernel, HIP graph) with and without the repair, against the
    plain per-problem loop (rollout, weights, update, repair calls per problem)."""
    import torch

    rep3 = dict(n_steps=10, step=0.05, objective=W.OBJ_TOTAL)
    p3 = [W.round_to_f32(p) for p in W.config3()]
    db3 = core.DeviceBatch(p3, dtype=torch.float32)
    pa = core.Plan(ctx, db3, M, C, seed, lam, repair=rep3, use_graph=True)
    pb = core.Plan(ctx, db3, M, C, seed, lam, use_graph=True)
    ta = _time(pa.launch, 20, 3, sync)
    tb = _time(pb.launch, 20, 3, sync)
    frac = _active_fraction(db3, pa.V_plus, pa.V_safe)
    dbs = [core.DeviceBatch([p], dtype=torch.float32, pid_base=b) for b, p in enumerate(p3)]

    def loop(repair):
        for d in dbs:
            S = core.rollout(ctx, d, M, C, seed)
            w, _ = core.weights(ctx, d, S, lam)
            Vp = core.update(ctx, d, M, C, seed, w)
            if repair:
                core.shield_repair(ctx, d, M, C, Vp, 10, 0.05, W.OBJ_TOTAL)

    tla = _time(lambda: loop(True), 5, 1, sync)
    tlb = _time(lambda: loop(False), 5, 1, sync)
    # the shield's own objective (Algorithm 1 hinge), which stops once V+ is safe
    pc = core.Plan(ctx, db3, M, C, seed, lam, repair=rep, use_graph=True)
    tc = _time(pc.launch, 20, 3, sync)
    frac_c = _active_fraction(db3, pc.V_plus, pc.V_safe)
    steps = sum(p.K * p.T for p in p3)
    out["c3_B64_K2048_T50"] = {
        "objective": "total cost + sum of squared DCBF violations, 10 steps x 0.05",
        "batched_with_repair_ms": ta * 1e3, "batched_without_repair_ms": tb * 1e3,
        "plain_loop_with_repair_ms": tla * 1e3, "plain_loop_without_repair_ms": tlb * 1e3,
        "speedup_with_repair": tla / ta, "batched_with_repair_rollout_steps_per_s": steps / ta,
        "shield_active_fraction": frac,
        "shield_objective": {"with_shield_ms": tc * 1e3, "shield_active_fraction": frac_c}}
    _log(f"  c3: {out['c3_B64_K2048_T50']}")
    for pl in (pa, pb, pc):
        pl.close()


def _form_c4_adjoint(ctx, core, W, M, C, lam, sync, out, seed):
    """Config 4's adjoint: the gradient of the free energy -lambda log sum exp(-S/lambda)
    (upstream g = the weights) at K = 65536, T = 100 with 64 obstacles, states recomputed
    from checkpoints; the adjoint kernel alone and rollout + weights + adjoint."""
    import torch

    p4 = W.round_to_f32(W.config4())
    db4 = core.DeviceBatch([p4], dtype=torch.float32)
    obj = dict(w_S=1.0, w_sq=0.0, w_lin=0.0, n_lin=0)
    S = core.rollout(ctx, db4, M, C, seed)
    w, _ = core.weights(ctx, db4, S, lam)
    gV = db4.new_V()
    t_adj = _time(lambda: core.rollout_backward(ctx, db4, M, C, seed, w, obj, out=gV), 10, 2, sync)

    def full():
        S2 = core.rollout(ctx, db4, M, C, seed, S=S)
        w2, _ = core.weights(ctx, db4, S2, lam)
        core.rollout_backward(ctx, db4, M, C, seed, w2, obj, out=gV)

    t_full = _time(full, 10, 2, sync)
    steps = p4.K * p4.T
    out["c4_free_energy_adjoint"] = {"adjoint_ms": t_adj * 1e3, "adjoint_rollout_steps_per_s": steps / t_adj,
                                     "rollout_weights_adjoint_ms": t_full * 1e3}
    _log(f"  c4 adjoint: {out['c4_free_energy_adjoint']}")


def _form_shield(ctx, core, W, M, C, rep, sync, out):
    """The shield alone on 64 violating problems (T = 50, spline tracks): Algorithm 1
    vs the projected L-BFGS variant, same steps and delta; time and the summed DCBF
    violation left (FP64 oracle objective of the device result)."""
    import torch

    import oracle

    probs = []
    for b in range(64):
        tr = W.spline_track(100 + b)
        V = W.test_sequences(1, 50, seed=300 + b, scale=0.8)[0]
        probs.append(W.round_to_f32(W.Problem(1, 50, tr, W.start_state(tr, vx=3.0 + (b % 3)), V, b, 0)))
    db = core.DeviceBatch(probs, dtype=torch.float32)
    before = np.mean([oracle.objective(W.MODEL, W.COST, p.track, p.x0, p.V, rep["objective"])[0] for p in probs])
    res = {"problems": 64, "T": 50, "steps": rep["n_steps"], "delta": rep["step"],
           "violation_before": float(before)}
    for method in ("gradient", "lbfgs"):
        def run():
            return core.shield_repair(ctx, db, M, C, db.V, rep["n_steps"], rep["step"], rep["objective"],
                                      method=method, memory=5)
        dt = _time(run, 50, 5, sync)
        Vs = db.controls(run())
        after = np.mean([oracle.objective(W.MODEL, W.COST, p.track, p.x0, Vs[b].astype(np.float64),
                                          rep["objective"])[0] for b, p in enumerate(probs)])
        res[method] = {"ms": dt * 1e3, "violation_after": float(after)}
    out["shield_B64_T50"] = res
    _log(f"  shield: {res}")


def _form_autotune(ctx, core, W, M, C, lam, sync, out, seed):
    """Autotuner table on the 512-problem ragged batch and on the headline shape
    (fused kernel alone, kernel-stamped events; no cache file)."""
    import torch

    from paper_2302_11719_amd import autotune

    for name, probs in (("ragged_B512", [W.round_to_f32(p) for p in W.config2()]),
                        ("headline_K4096_T50", [W.round_to_f32(W.config1(K=4096, T=50))])):
        db = core.DeviceBatch(probs, dtype=torch.float32)
        r = autotune.tune(ctx, db, M, C, seed, lam, reps=5, warmup=2, cache=None)
        default = core.Plan(ctx, db, M, C, seed, lam, use_graph=False)
        info = default.info()
        dms = []
        for i in range(7):
            default.launch_profiled()
            if i >= 2:
                dms.append(default.kernel_ms()[0])
        default.close()
        out[f"autotune_{name}"] = {"best": r.best, "best_kernel_ms": r.best_ms,
                                   "default": info, "default_kernel_ms": float(np.median(dms)),
                                   "candidates": len(r.table), "top5": r.table[:5], "worst": r.table[-1]}
        _log(f"  autotune {name}: best {r.best} {r.best_ms:.4f} ms; default {info} {np.median(dms):.4f} ms; "
             f"worst {r.table[-1]['kernel_ms']:.4f} ms over {len(r.table)} candidates")


def _form_sweep(ctx, out):
    """Closed-loop collision sweep (the paper's second experiment, on generated tracks):
    100 runs x 150 steps per cell, K in {64, 256, 1024}, T in {10, 20, 40}, three
    controllers; target speed 8 m/s on half width 0.9 m, disturbance 0.3."""
    from paper_2302_11719_amd import sweep

    t0 = time.perf_counter()
    rows = sweep.sweep(ctx, (64, 256, 1024), (10, 20, 40), runs=100, steps=150, seed=1, v_goal=8.0)
    out["sweep_collisions"] = {"runs": 100, "steps": 150, "v_goal": 8.0, "half_width": 0.9, "dist_sigma": 0.3,
                               "cells": rows, "wall_s": time.perf_counter() - t0}
    for r in rows:
        _log(f"  sweep K={r['K']} T={r['T']} {r['controller']}: collision rate {r['collision_rate']:.2f}, "
             f"{r['collisions_per_run']:.2f} collided steps/run, {r['ms_per_step']:.3f} ms/step")


def _form_curvilinear(ctx, core, W, M, C, sync, out, seed):
    """The eight-state curvilinear model (the paper's vehicle state, with wheel speeds):
    its rollout at K = 65536, T = 100 beside the Cartesian rollout of the same size on the
    same track (no obstacles), its free-energy adjoint at the same size, and one
    closed-loop Shield-MPPI iteration at K = 4096, T = 50 through the plain calls
    (rollout, weights, update, shield, plant step), called one by one and captured once
    in a HIP graph."""
    import torch

    K, T = 65536, 100
    p = W.round_to_f32(W.config1(K=K, T=T))
    db = core.DeviceBatch([p], dtype=torch.float32)
    S = db.new_S()
    t_cart = _time(lambda: core.rollout(ctx, db, M, C, seed, S=S), 20, 3, sync)
    kap, ds = W.curvature_table(p.track, 1024)
    WH = W.wheels_f32()
    pc = W.Problem(K, T, p.track, W.start_state_c8(3.0), p.V, 0, 0)
    dbc = core.DeviceBatch([W.round_to_f32(pc)], dtype=torch.float32)
    ct = core.CurvTrackArrays([(kap, ds)], [p.track.half_width])
    t_curv = _time(lambda: core.rollout_curvilinear(ctx, dbc, ct, M, WH, C, seed, S=S), 20, 3, sync)
    w, _ = core.weights(ctx, dbc, core.rollout_curvilinear(ctx, dbc, ct, M, WH, C, seed), W.LAMBDA)
    gV = dbc.new_V()
    obj = dict(w_S=1.0, w_sq=0.0, w_lin=0.0, n_lin=0)
    t_adj = _time(lambda: core.rollout_backward_curvilinear(ctx, dbc, ct, M, WH, C, seed, w, obj, out=gV), 10, 2,
                  sync)
    # closed loop: Algorithm 2 with Algorithm 1 through the plain calls
    Kl, Tl = 4096, 50
    pl = W.Problem(Kl, Tl, p.track, W.start_state_c8(3.0), np.zeros((Tl, 2)), 0, 0)
    dbl = core.DeviceBatch([W.round_to_f32(pl)], dtype=torch.float32)

    def loop_iter():
        Sl = core.rollout_curvilinear(ctx, dbl, ct, M, WH, C, seed)
        wl, _ = core.weights(ctx, dbl, Sl, W.LAMBDA)
        Vp = core.update(ctx, dbl, M, C, seed, wl)
        Vs = core.shield_repair_curvilinear(ctx, dbl, ct, M, WH, C, Vp, 10, 0.05, W.OBJ_SHIELD)
        core.execute_curvilinear(ctx, dbl, ct, M, WH, Vs, Vp)

    t_loop = _time(loop_iter, 50, 5, sync)
    # the shield with every one of its ten steps active (total cost + squared violations)
    Sl = core.rollout_curvilinear(ctx, dbl, ct, M, WH, C, seed)
    Vq = core.update(ctx, dbl, M, C, seed, core.weights(ctx, dbl, Sl, W.LAMBDA)[0])
    t_sh = _time(lambda: core.shield_repair_curvilinear(ctx, dbl, ct, M, WH, C, Vq, 10, 0.05, W.OBJ_TOTAL), 20, 3,
                 sync)
    g = _capture(loop_iter)
    t_graph = _time(g.replay, 50, 5, sync)
    del g
    out["curvilinear8_K65536_T100"] = {
        "rollout_ms": t_curv * 1e3, "rollout_steps_per_s": K * T / t_curv,
        "achieved_TFLOPs": FLOP_STEP_C8 * K * T / t_curv / 1e12,
        "free_energy_adjoint_ms": t_adj * 1e3,
        "cartesian_rollout_ms": t_cart * 1e3, "cartesian_rollout_steps_per_s": K * T / t_cart,
        "cartesian_achieved_TFLOPs": FLOP_STEP_POLY * K * T / t_cart / 1e12,
        "closed_loop_K4096_T50_ms_per_iter": t_loop * 1e3,
        "closed_loop_K4096_T50_graph_ms_per_iter": t_graph * 1e3,
        "shield_10_active_steps_T50_ms": t_sh * 1e3}
    _log(f"  curvilinear: {out['curvilinear8_K65536_T100']}")


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_closed_loop(W, K, T, lam, rep, threads, budget_s, max_it):
    import oracle

    p = W.config1(K=K, T=T)
    x, V = p.x0.copy(), p.V.copy()
    dist = W.disturbances(0, max_it)
    n_it = 0
    t0 = time.perf_counter()
    while True:
        r = oracle.mppi_iteration(W.MODEL, W.COST, p.track, x, V, K, 0, 0, n_it, lam, n_threads=threads)
        Vs = oracle.repair(W.MODEL, W.COST, p.track, x, r["V_plus"], rep["n_steps"], rep["step"], rep["objective"])
        x = oracle.execute(W.MODEL, x, Vs[0], dist[n_it])
        V = oracle.shift(r["V_plus"])
        n_it += 1
        el = time.perf_counter() - t0
        if el > budget_s or n_it >= max_it:
            return n_it, el


def _oracle_iteration_time(W, probs, lam, threads, repair=None):
    """Wall time of one oracle MPPI iteration over the given problems (rollout threaded
    over samples, then weights, update and optionally the repair, problem by problem)."""
    import oracle

    t0 = time.perf_counter()
    for b, p in enumerate(probs):
        r = oracle.mppi_iteration(W.MODEL, W.COST, p.track, p.x0, p.V, p.K, 0, b, p.it, lam, n_threads=threads)
        if repair:
            oracle.repair(W.MODEL, W.COST, p.track, p.x0, r["V_plus"], repair["n_steps"], repair["step"],
                          repair["objective"])
    return time.perf_counter() - t0


def oracle_configs(W, lam, cores):
    """The oracle timed on the other workloads (same inputs as the GPU forms): config 0
    whole (median of 5), config 2 once on all threads and on a sample of its problems on
    one thread, config 3 (with the 10-step repair) on all threads and on a sample on one
    thread, config 4 (64 obstacles) on all threads and on a sample of its samples on one
    thread.  Rates are rollout-steps per second of the sampled work."""
    import oracle

    res = {}
    p0 = W.config0()
    t_n = float(np.median([_oracle_iteration_time(W, [p0], lam, cores) for _ in range(5)]))
    t_1 = float(np.median([_oracle_iteration_time(W, [p0], lam, 1) for _ in range(5)]))
    st0 = p0.K * p0.T
    res["c0_fp64_K256_T20"] = {"ms_per_iter": t_n * 1e3, "rollout_steps_per_s": st0 / t_n,
                               "single_thread": {"ms_per_iter": t_1 * 1e3, "rollout_steps_per_s": st0 / t_1}}
    p2 = W.config2()
    st2 = sum(p.K * p.T for p in p2)
    t_n = _oracle_iteration_time(W, p2, lam, cores)
    sample = p2[::32]
    t_1 = _oracle_iteration_time(W, sample, lam, 1)
    st2s = sum(p.K * p.T for p in sample)
    res["c2_ragged_B512"] = {"ms_per_iter": t_n * 1e3, "rollout_steps_per_s": st2 / t_n,
                             "single_thread": {"rollout_steps_per_s": st2s / t_1, "problems": len(sample),
                                               "ms": t_1 * 1e3}}
    rep3 = dict(n_steps=10, step=0.05, objective=W.OBJ_TOTAL)
    p3 = W.config3()
    st3 = sum(p.K * p.T for p in p3)
    t_n = _oracle_iteration_time(W, p3, lam, cores, rep3)
    t_1 = _oracle_iteration_time(W, p3[:4], lam, 1, rep3)
    res["c3_B64_K2048_T50_repair"] = {"ms_per_iter": t_n * 1e3, "rollout_steps_per_s": st3 / t_n,
                                      "single_thread": {"problems": 4, "ms": t_1 * 1e3,
                                                        "ms_per_iter_64_extrapolated": 16 * t_1 * 1e3}}
    p4 = W.config4()
    t0 = time.perf_counter()
    oracle.rollout(W.MODEL, W.COST, p4.track, p4.x0, p4.V, p4.K, 0, 0, 0, want_eps=False, n_threads=cores)
    t_n = time.perf_counter() - t0
    ms = np.arange(0, p4.K, 16)
    t0 = time.perf_counter()
    oracle.rollout(W.MODEL, W.COST, p4.track, p4.x0, p4.V, 0, 0, 0, 0, want_eps=False, samples=ms)
    t_1 = time.perf_counter() - t0
    res["c4_K65536_T100_obs64_rollout"] = {"ms": t_n * 1e3, "rollout_steps_per_s": p4.K * p4.T / t_n,
                                           "single_thread": {"samples": len(ms),
                                                             "rollout_steps_per_s": len(ms) * p4.T / t_1}}
    return res


def cpu_baseline(W, K, T, lam, rep):
    """The FP64 oracle, as it stands, on a bounded sample of the headline workload:
    a few closed-loop iterations (rollout of all K samples, weights, update, shield,
    plant), with the rollout threaded over the host's cores, and the same again on
    one thread."""
    cores = min(os.cpu_count() or 1, 16)
    n_it, el = _oracle_closed_loop(W, K, T, lam, rep, cores, 10.0, 60)
    n1, el1 = _oracle_closed_loop(W, K, T, lam, rep, 1, 5.0, 60)
    return {"value": K * T * n_it / el, "unit": "rollout-steps/s", "cores": cores, "kind": "oracle",
            "ms_per_iter": 1e3 * el / n_it,
            "single_thread": {"value": K * T * n1 / el1, "ms_per_iter": 1e3 * el1 / n1, "iterations": n1},
            "cpu": _cpu_model(),
            "sample": f"{n_it} closed-loop iterations of the headline workload (K={K}, T={T}, shield on), "
                      f"FP64 oracle, rollout threaded over {cores} host threads; {n1} more on one thread",
            "other_configs": oracle_configs(W, lam, cores)}


if __name__ == "__main__":
    main()
