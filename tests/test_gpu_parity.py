"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (stated per check): FP64 device runs agree to rounding (1e-10
relative on costs); FP32 per-sample costs to 1e-4 relative (floor 1), weights
given identical costs to 1e-6, the update given identical weights to 1e-5, and
gradients to 1e-3 relative in norm.  Samples whose trajectory passes within
1e-3 of a collision-indicator switch are excluded from FP32 cost parity (the
indicator is discontinuous) and counted.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2302_11719_amd import core
from paper_2302_11719_amd import workloads as W

from gpu_helpers import band_mask, ctx, device_iteration, oracle_iteration, params, prep, ragged_problems, rel_err, say

pytestmark = pytest.mark.gpu
F32, F64 = torch.float32, torch.float64
BAND = 1e-3


def test_philox_words_bit_exact():
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2 ** 32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0
    key = (0xA4093822, 0x299F31D0)
    say("philox: 4096 counters")
    dev = core.debug_philox(ctx(), ctr, key)
    ref = np.stack([oracle.philox(c, key) for c in ctr])
    assert np.array_equal(dev, ref)


def test_c0_fp64_iteration():
    """K=256, T=20, circle track, FP64: costs, effective noise, weights, update."""
    p = W.config0()
    say("c0 fp64 K=256 T=20")
    d = device_iteration([p], F64, seed=0, lam=W.LAMBDA, want_eps=True)
    r = oracle_iteration(p, W.MODEL, W.COST, 0, W.LAMBDA)
    S = d["S"].cpu().numpy()
    assert rel_err(S, r["S"]).max() <= 1e-10
    eps = d["eps"].cpu().numpy()[:, :p.T]
    assert np.abs(eps - r["eps"]).max() <= 1e-12
    assert np.abs(d["w"].cpu().numpy() - r["w"]).max() <= 1e-10
    st = d["stats"].cpu().numpy()[0]
    assert st[0] == pytest.approx(r["stats"][0], rel=1e-12)
    assert st[1] == pytest.approx(r["stats"][1], abs=1e-9)
    assert st[2] == pytest.approx(r["stats"][2], rel=1e-9)
    assert st[3] == 0
    Vp = d["db"].controls(d["V_plus"])[0]
    assert np.abs(Vp - r["V_plus"]).max() <= 1e-10


@pytest.mark.parametrize("K,T", [(4096, 50), (1000, 33)])
def test_fp32_iteration_spline(K, T):
    """Single FP32 iteration on the spline track (K=4096, T=50 is the closed-loop shape)."""
    p = prep([W.config1(K=K, T=T)], F32)[0]
    p.V = W.round_to_f32(W.Problem(K, T, p.track, p.x0, W.test_sequences(1, T, 7, 0.3)[0])).V
    M, C = params(F32)
    say(f"fp32 spline K={K} T={T}")
    d = device_iteration([p], F32, seed=11, lam=W.LAMBDA, want_eps=True)
    r = oracle_iteration(p, M, C, 11, W.LAMBDA)
    S = d["S"].cpu().numpy().astype(np.float64)
    ok = band_mask(r["margin"], BAND, "", S, r["S"])
    assert ok.mean() > 0.95
    e = rel_err(S, r["S"])
    assert e[ok].max() <= 1e-4, e[ok].max()
    eps = d["eps"].cpu().numpy()[:, :T].astype(np.float64)
    assert np.abs(eps - r["eps"]).max() <= 2e-6
    # weights given identical costs
    w_ref, st_ref = oracle.weights(S, W.LAMBDA)
    w = d["w"].cpu().numpy().astype(np.float64)
    assert np.abs(w - w_ref).max() <= 1e-6
    assert abs(w.sum() - 1.0) <= 1e-5
    st = d["stats"].cpu().numpy()[0]
    assert st[0] == pytest.approx(st_ref[0], rel=1e-7)
    assert st[2] == pytest.approx(st_ref[2], rel=1e-4)
    # update given identical weights and the oracle's own effective noise
    Vp = d["db"].controls(d["V_plus"])[0]
    Vp_ref = oracle.update(p.V, w, r["eps"])
    assert np.abs(Vp - Vp_ref).max() <= 1e-5


@pytest.mark.parametrize("dtype", [F32, F64])
def test_ragged_batch(dtype):
    """Five problems of uneven K and T (ragged tails, K=1, T=1), circle and spline
    tracks, obstacles on one: per-sample costs and the update of every problem."""
    probs = prep(ragged_problems(), dtype)
    M, C = params(dtype)
    say(f"ragged batch {dtype}")
    d = device_iteration(probs, dtype, seed=5, lam=W.LAMBDA)
    Ss = d["db"].per_problem(d["S"])
    ws = d["db"].per_problem(d["w"])
    Vps = d["db"].controls(d["V_plus"])
    tol = 1e-4 if dtype == F32 else 1e-10
    for b, p in enumerate(probs):
        r = oracle_iteration(p, M, C, 5, W.LAMBDA)
        ok = band_mask(r["margin"], BAND if dtype == F32 else 0.0, f'problem {b}', Ss[b], r["S"], tol)
        e = rel_err(Ss[b], r["S"])
        assert e[ok].max() <= tol, (b, e[ok].max())
        Vp_ref = oracle.update(p.V, ws[b].astype(np.float64), r["eps"])
        assert np.abs(Vps[b] - Vp_ref).max() <= (1e-5 if dtype == F32 else 1e-12), b


def test_empty_problem_keeps_controls():
    probs = ragged_problems()
    probs[1].K = 0
    say("ragged batch with K=0")
    d = device_iteration(probs, F64, seed=1, lam=1.0)
    Vps = d["db"].controls(d["V_plus"])
    assert np.array_equal(Vps[1], probs[1].V)
    st = d["stats"].cpu().numpy()[1]
    assert np.isinf(st[0]) and st[3] == 0


@pytest.mark.parametrize("dtype", [F32, F64])
def test_invariants(dtype):
    """Zero noise returns the nominal control with equal costs; K=1 returns that
    sample; weights sum to one; V+ stays in the control box."""
    p = prep([W.config1(K=777, T=30)], dtype)[0]
    p.V = prep([W.Problem(777, 30, p.track, p.x0, W.test_sequences(1, 30, 3, 0.6)[0])], dtype)[0].V
    M, C = params(dtype)
    say(f"invariants {dtype}")
    d = device_iteration([p], dtype, seed=2, lam=W.LAMBDA, nominal=True)
    S = d["S"].cpu().numpy()
    assert np.all(S == S[0])
    Sn, _, _ = oracle.rollout(M, C, p.track, p.x0, p.V, 1, 0, 0, 0, nominal=True)
    assert rel_err(S[:1], Sn).max() <= (1e-4 if dtype == F32 else 1e-10)
    assert np.array_equal(d["db"].controls(d["V_plus"])[0], p.V.astype(np.float32 if dtype == F32 else np.float64))
    d = device_iteration([p], dtype, seed=2, lam=W.LAMBDA)
    w = d["w"].cpu().numpy().astype(np.float64)
    assert abs(w.sum() - 1.0) <= (1e-5 if dtype == F32 else 1e-12)
    Vp = d["db"].controls(d["V_plus"])[0]
    assert np.all(Vp >= np.array(M["u_lo"]) - 1e-6) and np.all(Vp <= np.array(M["u_hi"]) + 1e-6)
    p1 = W.Problem(1, 30, p.track, p.x0, p.V, 0, 0)
    d = device_iteration([p1], dtype, seed=2, lam=W.LAMBDA)
    z = oracle.normals(2, 0, 0, 0, 30) * np.array(C["sigma"])
    Vp = d["db"].controls(d["V_plus"])[0]
    assert np.abs(Vp - np.clip(p.V + z, M["u_lo"], M["u_hi"])).max() <= (2e-6 if dtype == F32 else 1e-13)


def _grad_problem(dtype, K=6, T=20, n_obs=16):
    p = W.config4(K=K, T=T, n_obs=n_obs)
    p.V = W.test_sequences(1, T, seed=9, scale=0.5)[0]
    return prep([p], dtype)[0]


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("obj", ["total", "shield", "mixed"])
def test_backward_vs_oracle(dtype, obj):
    """Adjoint gradient sum_m g_m dL_m/dV vs the oracle's dual-number gradient."""
    objective = {"total": W.OBJ_TOTAL, "shield": W.OBJ_SHIELD,
                 "mixed": dict(w_S=0.5, w_sq=2.0, w_lin=1.0, n_lin=12)}[obj]
    p = _grad_problem(dtype)
    M, C = params(dtype)
    db = core.DeviceBatch([p], dtype=dtype)
    g = np.linspace(0.5, 1.5, p.K)
    say(f"backward {dtype} {obj} K={p.K} T={p.T}")
    gV = core.rollout_backward(ctx(), db, M, C, 4, torch.as_tensor(g, dtype=dtype, device="cuda"), objective)
    torch.cuda.synchronize()
    gV = db.controls(gV)[0]
    ref = np.zeros((p.T, 2))
    for m in range(p.K):
        eps = oracle.normals(4, p.pid, p.it, m, p.T) * np.array(C["sigma"])
        ref += g[m] * oracle.gradient_dual(M, C, p.track, p.x0, p.V, objective, eps)
    err = np.linalg.norm(gV - ref) / max(np.linalg.norm(ref), 1e-30)
    tol = 1e-3 if dtype == F32 else 1e-9
    assert err <= tol, err
    assert np.abs(gV - ref).max() <= tol * np.abs(ref).max()


def test_backward_central_differences_fp64():
    """FP64 central differences (h = 1e-6) on 8 seeded sequences, nominal trajectory,
    total cost plus squared violations."""
    M, C = W.MODEL, W.COST
    tr = W.spline_track(0)
    x0 = W.start_state(tr)
    seqs = W.test_sequences(8, 50, seed=3, scale=0.5)
    probs = [W.Problem(1, 50, tr, x0, V, 0, 0) for V in seqs]
    db = core.DeviceBatch(probs, dtype=F64)
    say("backward vs FD fp64, 8 sequences T=50")
    gV = core.rollout_backward(ctx(), db, M, C, 0, torch.ones(8, dtype=F64, device="cuda"), W.OBJ_TOTAL,
                               nominal=True)
    torch.cuda.synchronize()
    checked = 0
    for b, V in enumerate(seqs):
        fd, valid = oracle.gradient_fd(M, C, tr, x0, V, W.OBJ_TOTAL, None, 1e-6)
        g = db.controls(gV)[b]
        scale = np.abs(fd[valid]).max()
        assert np.abs(g - fd)[valid].max() <= 1e-3 * scale
        checked += valid.sum()
    assert checked >= 8 * 100 * 0.9


def test_autograd_function():
    from paper_2302_11719_amd.autograd import SmppiRolloutCost

    p = _grad_problem(F64, K=5, T=12, n_obs=0)
    M, C = params(F64)
    db = core.DeviceBatch([p], dtype=F64)
    V = db.V.clone().requires_grad_(True)
    say("autograd function fp64")
    S = SmppiRolloutCost.apply(V, ctx(), db, M, C, 8, False)
    g = torch.arange(1, p.K + 1, dtype=F64, device="cuda")
    (S * g).sum().backward()
    ref = np.zeros((p.T, 2))
    for m in range(p.K):
        eps = oracle.normals(8, p.pid, p.it, m, p.T) * np.array(C["sigma"])
        ref += (m + 1) * oracle.gradient_dual(M, C, p.track, p.x0, p.V, dict(w_S=1.0, w_sq=0.0, w_lin=0.0,
                                                                             n_lin=0), eps)
    got = db.controls(V.grad)[0]
    assert np.abs(got - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("method", ["gradient", "lbfgs"])
@pytest.mark.parametrize("dtype", [F32, F64])
def test_shield_repair_vs_oracle(dtype, method):
    """Algorithm 1 (10 projected steps, delta = 0.05) on the nominal trajectory, and the
    projected L-BFGS variant (memory 5) with the same steps and delta."""
    tr_c = W.circle_track(10.0, 1.0)
    probs = [W.Problem(1, 30, tr_c, W.start_state(tr_c, vx=4.0), np.tile([-0.2, 0.6], (30, 1)), 0, 0)]
    for b in range(3):
        tr = W.spline_track(b)
        probs.append(W.Problem(1, 25 + 5 * b, tr, W.start_state(tr, vx=3.0 + b),
                               W.test_sequences(1, 25 + 5 * b, seed=20 + b, scale=0.8)[0], b + 1, 0))
    probs = prep(probs, dtype)
    M, C = params(dtype)
    db = core.DeviceBatch(probs, dtype=dtype)
    say(f"repair {dtype} {method}")
    Vs = core.shield_repair(ctx(), db, M, C, db.V, 10, 0.05, W.OBJ_SHIELD, method=method, memory=5)
    torch.cuda.synchronize()
    assert ctx().device_errors() == 0
    got = db.controls(Vs)
    for b, p in enumerate(probs):
        ref = oracle.repair(M, C, p.track, p.x0, p.V, 10, 0.05, W.OBJ_SHIELD, method=method, memory=5)
        tol = 1e-3 * max(np.linalg.norm(p.V), 1.0) if dtype == F32 else 1e-9
        assert np.abs(got[b] - ref).max() <= tol, (b, np.abs(got[b] - ref).max())
    before, _ = oracle.objective(M, C, probs[0].track, probs[0].x0, probs[0].V, W.OBJ_SHIELD)
    after, _ = oracle.objective(M, C, probs[0].track, probs[0].x0, got[0].astype(np.float64), W.OBJ_SHIELD)
    assert after < before


def test_execute_and_warm_start():
    probs = ragged_problems()
    M, C = params(F64)
    db = core.DeviceBatch(probs, dtype=F64)
    Vp = db.V.clone() * 0.5
    dist = torch.as_tensor(W.disturbances(0, 3 * db.B).reshape(3, db.B, 2), dtype=F64, device="cuda")
    x_before = db.x0.cpu().numpy().reshape(-1, 6)
    it_before = db.iter.cpu().numpy()
    say("execute fp64")
    core.execute(ctx(), db, M, Vp, Vp, dist.reshape(-1), 3)
    torch.cuda.synchronize()
    x_after = db.x0.cpu().numpy().reshape(-1, 6)
    Vs = db.controls(db.V)
    Vp_l = db.controls(Vp)
    dnp = dist.cpu().numpy()
    for b, p in enumerate(probs):
        d = dnp[it_before[b], b] if it_before[b] < 3 else None
        ref = oracle.execute(M, x_before[b], Vp_l[b][0], d)
        assert np.abs(x_after[b] - ref).max() <= 1e-12
        assert np.array_equal(Vs[b], oracle.shift(Vp_l[b]))
    assert np.array_equal(db.iter.cpu().numpy(), it_before + 1)


def test_device_error_flags():
    """A batch whose declared t_max is smaller than a problem's horizon: the kernel's own
    bounds check skips the problem and raises the flag; nothing else is written."""
    probs = ragged_problems()
    M, C = params(F32)
    db = core.DeviceBatch(probs, dtype=F32)
    db.batch.t_max = 10  # problems 0 and 2 have T = 21 and 37
    S = torch.full((db.sum_K,), -7.0, device="cuda")
    say("device error flags")
    core.rollout(ctx(), db, M, C, 0, S=S)
    flags = ctx().device_errors()
    assert flags & 1
    Ss = db.per_problem(S)
    assert np.all(Ss[0] == -7.0) and np.all(Ss[2] == -7.0)
    assert np.all(Ss[1] != -7.0)
