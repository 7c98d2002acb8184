"""GPU parity of the eight-state curvilinear model (the paper's vehicle state with
wheel speeds) against the FP64 oracle: sampled rollout, the weights and update it
shares with the Cartesian path, the K-sample adjoint, the shield of Algorithm 1
and a teacher-forced closed loop (rollout, weights, update, shield, plant step)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
from paper_2302_11719_amd import core
from paper_2302_11719_amd import workloads as W

from gpu_helpers import band_mask, ctx, params, rel_err, say

pytestmark = pytest.mark.gpu
F32, F64 = torch.float32, torch.float64
BAND = 1e-3
OBJ_MIXED = dict(w_S=0.5, w_sq=2.0, w_lin=1.0, n_lin=12)


def _r32(a, dtype):
    a = np.asarray(a, dtype=np.float64)
    return a.astype(np.float32).astype(np.float64) if dtype == F32 else a


def _problems(dtype, specs):
    """specs: (track, table points, K, T, x0, V seed, V scale) per problem."""
    probs, tables, widths = [], [], []
    for b, (tr, n, K, T, x0, vseed, vscale) in enumerate(specs):
        kap, ds = W.curvature_table(tr, n)
        kap, ds = _r32(kap, dtype), float(_r32(ds, dtype))
        V = _r32(W.test_sequences(1, T, seed=vseed, scale=vscale)[0], dtype)
        probs.append(W.Problem(K, T, W.circle_track(10.0, 1.0), _r32(x0, dtype), V, b, b + 1))
        tables.append((kap, ds))
        widths.append(float(_r32(tr.half_width, dtype)))
    return probs, tables, widths


def _standard(dtype, K0=None):
    return _problems(dtype, [
        (W.spline_track(0), 1024, K0 or (4096 if dtype == F32 else 256), 50, W.start_state_c8(3.0, 0.1, 0.05), 40, 0.4),
        (W.spline_track(1), 512, 300, 23, W.start_state_c8(4.0, -0.2, -0.1, 12.0) + np.r_[0, 0.1, 0, 2, -3, 0, 0, 0],
         41, 0.5),
        (W.circle_track(10.0, 1.0), 256, 65, 7, W.start_state_c8(2.5, 0.0, 0.0, 1.0) + np.r_[0, 0, 0.1, 0, 0, 0, 0, 0],
         42, 0.4)])


def _device(probs, tables, widths, dtype):
    db = core.DeviceBatch(probs, dtype=dtype)
    ct = core.CurvTrackArrays(tables, widths, dtype=dtype)
    return db, ct


def _wheels(dtype):
    return W.wheels_f32() if dtype == F32 else dict(W.WHEELS)


@pytest.mark.parametrize("dtype", [F32, F64])
def test_c8_rollout_vs_oracle(dtype):
    probs, tables, widths = _standard(dtype)
    M, C = params(dtype)
    WH = _wheels(dtype)
    db, ct = _device(probs, tables, widths, dtype)
    say(f"c8 rollout {dtype}")
    S, eps = core.rollout_curvilinear(ctx(), db, ct, M, WH, C, 6, want_eps=True)
    torch.cuda.synchronize()
    assert ctx().device_errors() == 0
    Ss = db.per_problem(S)
    k0 = 0
    for b, p in enumerate(probs):
        kap, ds = tables[b]
        Sr, er, mg = oracle.rollout_c8(M, WH, C, kap, ds, widths[b], p.x0, p.V, p.K, 6, b, p.it)
        ok = band_mask(mg, BAND if dtype == F32 else 0.0, f'problem {b}', Ss[b], Sr, 1e-4 if dtype == F32 else 1e-10)
        assert ok.mean() > 0.9
        e = rel_err(Ss[b], Sr)
        assert e[ok].max() <= (1e-4 if dtype == F32 else 1e-10), (b, e[ok].max())
        ed = eps[k0:k0 + p.K, :p.T].cpu().numpy().astype(np.float64)
        assert np.abs(ed - er).max() <= (2e-6 if dtype == F32 else 1e-12)
        k0 += p.K


def test_c8_mppi_iteration_fp64():
    """Weights and update of the curvilinear costs (calls shared with the Cartesian model)."""
    probs, tables, widths = _standard(F64)
    M, C = params(F64)
    db, ct = _device(probs, tables, widths, F64)
    say("c8 MPPI iteration fp64")
    S = core.rollout_curvilinear(ctx(), db, ct, M, W.WHEELS, C, 8)
    w, _ = core.weights(ctx(), db, S, W.LAMBDA)
    Vp = core.update(ctx(), db, M, C, 8, w)
    torch.cuda.synchronize()
    Vps = db.controls(Vp)
    for b, p in enumerate(probs):
        kap, ds = tables[b]
        Sr, er, _ = oracle.rollout_c8(M, W.WHEELS, C, kap, ds, widths[b], p.x0, p.V, p.K, 8, b, p.it)
        wr, _ = oracle.weights(Sr, W.LAMBDA)
        assert np.abs(Vps[b] - oracle.update(p.V, wr, er)).max() <= 1e-9


def _sparse_g(K, n, rng, dtype):
    g = np.zeros(K)
    idx = np.unique(np.concatenate([np.linspace(0, K - 1, n).astype(int), [K - 1]]))
    g[idx] = rng.uniform(0.5, 1.5, size=len(idx)) * rng.choice([-1.0, 1.0], size=len(idx))
    return _r32(g, dtype)


def _oracle_grads(M, WH, C, probs, tables, widths, seed, gs, obj):
    sig = np.array(C["sigma"])
    jobs = [(b, int(m)) for b in range(len(probs)) for m in np.nonzero(gs[b])[0]]

    def one(job):
        b, m = job
        p = probs[b]
        kap, ds = tables[b]
        eps = oracle.normals(seed, b, p.it, m, p.T) * sig
        return b, gs[b][m] * oracle.gradient_dual_c8(M, WH, C, kap, ds, widths[b], p.x0, p.V, obj, eps)

    out = [np.zeros((p.T, 2)) for p in probs]
    with ThreadPoolExecutor(16) as ex:
        for b, g in ex.map(one, jobs):
            out[b] += g
    return out


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("obj", ["total", "mixed"])
def test_c8_backward_vs_oracle(dtype, obj):
    """K-sample adjoint with recomputed states on 2-64 workgroups per problem against the
    oracle's dual-number gradient (samples with nonzero upstream gradient)."""
    objective = W.OBJ_TOTAL if obj == "total" else OBJ_MIXED
    probs, tables, widths = _standard(dtype, K0=4096)
    M, C = params(dtype)
    WH = _wheels(dtype)
    db, ct = _device(probs, tables, widths, dtype)
    rng = np.random.default_rng(4)
    gs = [_sparse_g(p.K, 10, rng, dtype) for p in probs]
    say(f"c8 backward {dtype} {obj}")
    gV = core.rollout_backward_curvilinear(ctx(), db, ct, M, WH, C, 9,
                                           torch.as_tensor(np.concatenate(gs), dtype=dtype, device="cuda"), objective)
    torch.cuda.synchronize()
    assert ctx().device_errors() == 0
    ref = _oracle_grads(M, WH, C, probs, tables, widths, 9, gs, objective)
    got = db.controls(gV)
    tol = 1e-3 if dtype == F32 else 1e-9
    for b in range(len(probs)):
        err = np.linalg.norm(got[b] - ref[b]) / max(np.linalg.norm(ref[b]), 1e-30)
        emax = np.abs(got[b] - ref[b]).max() / max(np.abs(ref[b]).max(), 1e-30)
        say(f"  problem {b} K={probs[b].K}: rel err {err:.2e}")
        assert err <= tol and emax <= tol, (b, err, emax)


def _shield_problems(dtype):
    """Starts heading off the track so that the controls violate the DCBF condition."""
    return _problems(dtype, [
        (W.spline_track(2), 1024, 1, 30, W.start_state_c8(5.0, 0.4, 0.5), 50, 0.3),
        (W.spline_track(3), 512, 1, 25, W.start_state_c8(4.0, -0.5, -0.4, 20.0), 51, 0.3),
        (W.circle_track(10.0, 1.0), 256, 1, 20, W.start_state_c8(4.5, 0.6, 0.45), 52, 0.5)])


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("obj", ["shield", "total"])
def test_c8_shield_vs_oracle(dtype, obj):
    objective = W.OBJ_SHIELD if obj == "shield" else W.OBJ_TOTAL
    probs, tables, widths = _shield_problems(dtype)
    M, C = params(dtype)
    WH = _wheels(dtype)
    db, ct = _device(probs, tables, widths, dtype)
    say(f"c8 shield {dtype} {obj}")
    Vs = core.shield_repair_curvilinear(ctx(), db, ct, M, WH, C, db.V, 10, 0.05, objective)
    torch.cuda.synchronize()
    assert ctx().device_errors() == 0
    got = db.controls(Vs)
    for b, p in enumerate(probs):
        kap, ds = tables[b]
        before, _ = oracle.objective_c8(M, WH, C, kap, ds, widths[b], p.x0, p.V, objective)
        ref = oracle.repair_c8(M, WH, C, kap, ds, widths[b], p.x0, p.V, 10, 0.05, objective)
        tol = 1e-3 * max(np.linalg.norm(p.V), 1.0) if dtype == F32 else 1e-9
        assert np.abs(got[b] - ref).max() <= tol, (b, np.abs(got[b] - ref).max())
        if obj == "shield":
            assert before > 0.0
            after, _ = oracle.objective_c8(M, WH, C, kap, ds, widths[b], p.x0, got[b].astype(np.float64), objective)
            assert after < before


def test_c8_closed_loop_teacher_forced():
    """Algorithm 2 with Algorithm 1 on the curvilinear model (FP32, K = 2048, T = 40): four
    receding-horizon steps of rollout, weights, update, shield and the disturbed plant step
    through the C ABI, each checked against the oracle from the device's own state; the
    start heads off the track so that the shield acts."""
    probs, tables, widths = _problems(F32, [(W.spline_track(4), 1024, 2048, 40, W.start_state_c8(5.0, 0.4, 0.5),
                                             60, 0.2)])
    probs[0].V = np.zeros((40, 2))
    M, C = params(F32)
    WH = _wheels(F32)
    db, ct = _device(probs, tables, widths, F32)
    kap, ds = tables[0]
    dist_np = (W.disturbances(3, 8) * 0.5).astype(np.float32)
    dist = torch.as_tensor(dist_np.reshape(8, 1, 2), device="cuda")
    fired = 0
    for k in range(4):
        x_b = db.x0.cpu().numpy().astype(np.float64)
        V_b = db.controls(db.V)[0].astype(np.float64)
        it_b = int(db.iter.item())
        say(f"c8 closed loop step {k}")
        S = core.rollout_curvilinear(ctx(), db, ct, M, WH, C, 0)
        w, _ = core.weights(ctx(), db, S, W.LAMBDA)
        Vp = core.update(ctx(), db, M, C, 0, w)
        Vs = core.shield_repair_curvilinear(ctx(), db, ct, M, WH, C, Vp, 10, 0.05, W.OBJ_SHIELD)
        core.execute_curvilinear(ctx(), db, ct, M, WH, Vs, Vp, dist.reshape(-1), 8)
        torch.cuda.synchronize()
        assert ctx().device_errors() == 0
        Sn = S.cpu().numpy().astype(np.float64)
        S_ref, eps, margin = oracle.rollout_c8(M, WH, C, kap, ds, widths[0], x_b, V_b, 2048, 0, 0, it_b)
        ok = band_mask(margin, BAND, f'step {k}', Sn, S_ref)
        assert rel_err(Sn, S_ref)[ok].max() <= 1e-4
        w_ref, _ = oracle.weights(Sn, W.LAMBDA)
        Vpn = db.controls(Vp)[0].astype(np.float64)
        assert np.abs(Vpn - oracle.update(V_b, w_ref, eps)).max() <= 1e-5
        Vsn = db.controls(Vs)[0].astype(np.float64)
        Vs_ref = oracle.repair_c8(M, WH, C, kap, ds, widths[0], x_b, Vpn, 10, 0.05, W.OBJ_SHIELD)
        assert np.abs(Vsn - Vs_ref).max() <= 1e-3 * max(1.0, np.linalg.norm(Vpn))
        fired += int(not np.array_equal(Vsn, Vpn))
        x_ref = oracle.execute_c8(M, WH, kap, ds, x_b, Vsn[0], dist_np[it_b])
        assert np.abs(db.x0.cpu().numpy() - x_ref).max() <= 1e-4 * max(1.0, np.abs(x_ref).max())
        assert np.array_equal(db.controls(db.V)[0], oracle.shift(Vpn).astype(np.float32))
    say(f"  the shield changed V+ in {fired} of 4 steps")
    assert fired >= 1
