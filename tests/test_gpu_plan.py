"""GPU parity of the batched persistent plan (fused rollout + split softmax +
update, shield, execute; HIP graph) against the plain path and the oracle,
including sampled parity at the full workload sizes."""
import numpy as np
import pytest
import torch

import oracle
from paper_2302_11719_amd import core
from paper_2302_11719_amd import workloads as W

from gpu_helpers import band_mask, ctx, oracle_iteration, params, prep, ragged_problems, rel_err, say

pytestmark = pytest.mark.gpu
F32 = torch.float32
BAND = 1e-3


def _plain(db, M, C, seed, lam):
    c = ctx()
    S = core.rollout(c, db, M, C, seed)
    w, stats = core.weights(c, db, S, lam)
    Vp = core.update(c, db, M, C, seed, w)
    return S, w, stats, Vp


@pytest.mark.parametrize("block,tile,pipeline", [(256, 256, -1), (64, 128, -1), (128, 512, -1), (512, 512, -1),
                                                 (0, 0, 1)])
def test_plan_matches_plain_path(block, tile, pipeline):
    """Plan (fused persistent kernel; pipeline = 1 is the four-wave latency mode) against
    the plain per-call kernels and the oracle.  Tile mode runs the plain rollout's
    arithmetic (costs to 1e-6); the latency mode integrates the velocity part of RK4 in
    another evaluation order (stage factors folded into per-step coefficients) and sums
    the cost in partial sums, so its costs match the plain rollout's to the per-sample
    cost bar, 1e-4."""
    probs = prep(ragged_problems(), F32)
    M, C = params(F32)
    db = core.DeviceBatch(probs, dtype=F32)
    say(f"plan vs plain block={block} tile={tile} pipeline={pipeline}")
    S, w, stats, Vp = _plain(db, M, C, 5, W.LAMBDA)
    plan = core.Plan(ctx(), db, M, C, 5, W.LAMBDA, block=block, tile=tile, use_graph=False, pipeline=pipeline)
    plan.launch()
    torch.cuda.synchronize()
    assert ctx().device_errors() == 0
    err = float(rel_err(plan.S.cpu().numpy(), S.cpu().numpy().astype(np.float64)).max())
    assert err <= (1e-6 if pipeline < 0 else 1e-4), err
    ps, st = plan.stats.cpu().numpy().reshape(-1, 4), stats.cpu().numpy()
    if pipeline < 0:  # identical costs: V+ and the minimum agree to reduction order
        assert np.abs(plan.V_plus.cpu().numpy() - Vp.cpu().numpy()).max() <= 2e-5
        assert np.allclose(ps[:, 0], st[:, 0], rtol=1e-6)
    assert np.allclose(ps[:, 2], st[:, 2], rtol=1e-3)
    assert np.array_equal(ps[:, 3], st[:, 3])
    # and the oracle, problem by problem (V+ given the device costs)
    Ss = db.per_problem(plan.S)
    Vps = db.controls(plan.V_plus)
    for b, p in enumerate(probs):
        r = oracle_iteration(p, M, C, 5, W.LAMBDA)
        ok = band_mask(r["margin"], BAND, f'problem {b}', Ss[b], r["S"])
        assert rel_err(Ss[b], r["S"])[ok].max() <= 1e-4
        w_ref, _ = oracle.weights(Ss[b].astype(np.float64), W.LAMBDA)
        assert np.abs(Vps[b] - oracle.update(p.V, w_ref, r["eps"])).max() <= 1e-5


def test_plan_graph_replays_match_eager_plan():
    """Closed loop on the device: 4 graph replays (with eager work and synchronisations
    in between) equal 4 launches of the same plan without a graph."""
    probs = prep(ragged_problems(), F32)
    M, C = params(F32)
    dist = torch.as_tensor(W.disturbances(1, 8 * len(probs)).reshape(-1), dtype=F32, device="cuda")
    rep = dict(n_steps=3, step=0.05, objective=W.OBJ_SHIELD)
    dbs = [core.DeviceBatch(probs, dtype=F32) for _ in range(2)]
    # separate shield kernel: the launch has two kernels, so the first plan is a graph
    plans = [core.Plan(ctx(), dbs[i], M, C, 9, W.LAMBDA, repair=rep, execute=True, dist=dist.view(8, -1),
                       use_graph=(i == 0), fuse_shield=-1) for i in range(2)]
    for step in range(4):
        say(f"graph replay {step}")
        for pl in plans:
            pl.launch()
            torch.cuda.synchronize()
            _ = torch.zeros(1000, device="cuda").sum().item()  # eager work between replays
        for name in ("x0", "V", "iter"):
            assert torch.equal(getattr(dbs[0], name), getattr(dbs[1], name)), (step, name)
        assert torch.equal(plans[0].V_safe, plans[1].V_safe)
        assert torch.equal(plans[0].S, plans[1].S)
    assert ctx().device_errors() == 0
    assert np.array_equal(dbs[0].iter.cpu().numpy(), np.arange(1, 6) + 4)


@pytest.mark.parametrize("fuse", [-1, 1])
def test_profiled_launch_matches_and_times(fuse):
    """The profiled launch (events between the stages, kernel-stamped events on the
    fused and shield kernels) computes exactly what the ordinary launch computes, and
    its kernel-only durations are positive and within the stage durations (the shield's
    is 0 when it runs inside the fused launch)."""
    probs = prep(ragged_problems(), F32)
    M, C = params(F32)
    rep = dict(n_steps=3, step=0.05, objective=W.OBJ_SHIELD)
    dbs = [core.DeviceBatch(probs, dtype=F32) for _ in range(2)]
    plans = [core.Plan(ctx(), dbs[i], M, C, 4, W.LAMBDA, repair=rep, execute=True, use_graph=False,
                       fuse_shield=fuse) for i in range(2)]
    for step in range(3):
        say(f"profiled launch {step}")
        plans[0].launch()
        plans[1].launch_profiled()
        torch.cuda.synchronize()
        f, r, _ = plans[1].stage_ms()
        kf, kr = plans[1].kernel_ms()
        assert 0.0 < kf <= f + 1e-3, (f, kf)
        assert (0.0 < kr <= r + 1e-3) if fuse == -1 else kr == 0.0, (r, kr)
        for name in ("x0", "V", "iter"):
            assert torch.equal(getattr(dbs[0], name), getattr(dbs[1], name)), (step, name)
        assert torch.equal(plans[0].V_safe, plans[1].V_safe)
    assert ctx().device_errors() == 0


def test_default_fuses_the_shield_only_in_latency_mode():
    """fuse_shield = 0 runs the shield inside the launch in latency mode and as its own
    kernel in tile mode (the profiled launch times a shield kernel only when there is
    one); both give what the explicit choices give, bit for bit."""
    probs = prep(ragged_problems(), F32)
    M, C = params(F32)
    rep = dict(n_steps=3, step=0.05, objective=W.OBJ_SHIELD)
    for pipeline, block, fused in ((1, 0, True), (-1, 256, False)):
        say(f"default shield fusion pipeline={pipeline}")
        dbs = [core.DeviceBatch(probs, dtype=F32) for _ in range(2)]
        pd = core.Plan(ctx(), dbs[0], M, C, 5, W.LAMBDA, repair=rep, use_graph=False, pipeline=pipeline, block=block)
        pe = core.Plan(ctx(), dbs[1], M, C, 5, W.LAMBDA, repair=rep, use_graph=False, pipeline=pipeline, block=block,
                       fuse_shield=1 if fused else -1)
        pd.launch_profiled()
        pe.launch()
        torch.cuda.synchronize()
        assert (pd.kernel_ms()[1] == 0.0) == fused
        assert torch.equal(pd.V_safe, pe.V_safe) and torch.equal(pd.V_plus, pe.V_plus)
        pd.close()
        pe.close()
    assert ctx().device_errors() == 0


@pytest.mark.parametrize("pipeline,block,method", [(1, 0, "gradient"), (-1, 256, "gradient"), (-1, 128, "gradient"),
                                                   (-1, 64, "gradient"), (1, 0, "lbfgs"), (-1, 256, "lbfgs")])
def test_fused_shield_matches_separate_shield_kernel(pipeline, block, method):
    """Shield and execute run by the combining workgroup inside the fused launch equal
    the separate shield kernel bit for bit, over three closed-loop launches (blocks of
    64 and 128 threads have fewer than three waves, so they always use the separate
    kernel)."""
    probs = prep(ragged_problems(), F32)
    M, C = params(F32)
    dist = torch.as_tensor(W.disturbances(2, 8 * len(probs)).reshape(-1), dtype=F32, device="cuda")
    rep = dict(n_steps=4, step=0.05, objective=W.OBJ_SHIELD, method=method, memory=3)
    dbs = [core.DeviceBatch(probs, dtype=F32) for _ in range(2)]
    plans = [core.Plan(ctx(), dbs[i], M, C, 11, W.LAMBDA, repair=rep, execute=True, dist=dist.view(8, -1),
                       use_graph=False, pipeline=pipeline, block=block, fuse_shield=(1 if i == 0 else -1))
             for i in range(2)]
    for step in range(3):
        say(f"fused shield pipeline={pipeline} block={block} {method} step {step}")
        for pl in plans:
            pl.launch()
        torch.cuda.synchronize()
        assert torch.equal(plans[0].V_plus, plans[1].V_plus), step
        assert torch.equal(plans[0].V_safe, plans[1].V_safe), step
        for name in ("x0", "V", "iter"):
            assert torch.equal(getattr(dbs[0], name), getattr(dbs[1], name)), (step, name)
    assert ctx().device_errors() == 0


def test_closed_loop_teacher_forced_c1():
    """Config-1 shape (K=4096, T=50): 4 receding-horizon steps through the graph plan with
    the shield and the disturbed plant; every step checked against the oracle from the
    device's own state (teacher forcing)."""
    p = prep([W.config1()], F32)[0]
    M, C = params(F32)
    db = core.DeviceBatch([p], dtype=F32)
    dist_np = W.disturbances(0, 8).astype(np.float32)
    dist = torch.as_tensor(dist_np.reshape(-1), device="cuda")
    rep = dict(n_steps=10, step=0.05, objective=W.OBJ_SHIELD)
    plan = core.Plan(ctx(), db, M, C, 0, W.LAMBDA, repair=rep, execute=True, dist=dist.view(8, 1, 2),
                     use_graph=True)
    for k in range(4):
        x_b = db.x0.cpu().numpy().astype(np.float64)
        V_b = db.controls(db.V)[0].astype(np.float64)
        it_b = int(db.iter.item())
        say(f"closed loop step {k} it={it_b}")
        plan.launch()
        torch.cuda.synchronize()
        S = plan.S.cpu().numpy().astype(np.float64)
        S_ref, eps, margin = oracle.rollout(M, C, p.track, x_b, V_b, p.K, 0, 0, it_b)
        ok = band_mask(margin, BAND, f'step {k}', S, S_ref)
        assert rel_err(S, S_ref)[ok].max() <= 1e-4
        w_ref, _ = oracle.weights(S, W.LAMBDA)
        Vp = db.controls(plan.V_plus)[0].astype(np.float64)
        assert np.abs(Vp - oracle.update(V_b, w_ref, eps)).max() <= 1e-5
        Vs = db.controls(plan.V_safe)[0].astype(np.float64)
        Vs_ref = oracle.repair(M, C, p.track, x_b, Vp, 10, 0.05, W.OBJ_SHIELD)
        assert np.abs(Vs - Vs_ref).max() <= 1e-3 * max(1.0, np.linalg.norm(Vp))
        x_ref = oracle.execute(M, x_b, Vs[0], dist_np[it_b])
        assert np.abs(db.x0.cpu().numpy() - x_ref).max() <= 1e-5
        assert np.array_equal(db.controls(db.V)[0], oracle.shift(Vp).astype(np.float32))
    assert ctx().device_errors() == 0


def _sampled(p, S_dev, M, C, seed, n, rng):
    ms = np.sort(rng.choice(p.K, size=min(n, p.K), replace=False))
    S_ref, _, margin = oracle.rollout(M, C, p.track, p.x0, p.V, 0, seed, p.pid, p.it, want_eps=False,
                                      samples=ms)
    ok = band_mask(margin, BAND, 'sampled', S_dev[ms], S_ref)
    return rel_err(S_dev[ms], S_ref)[ok], (~ok).sum()


def test_full_size_config2_sampled():
    """512 ragged problems (K log-uniform in [256, 16384], T in [20, 100]) in the plan's
    launch configuration: sampled per-sample costs vs the oracle, and V+ vs the plain
    weights + update kernels applied to the plan's own costs."""
    probs = prep(W.config2(), F32)
    M, C = params(F32)
    db = core.DeviceBatch(probs, dtype=F32)
    say(f"config2 full: B={db.B} sum K={db.sum_K}")
    plan = core.Plan(ctx(), db, M, C, 0, W.LAMBDA, use_graph=True)
    plan.launch()
    torch.cuda.synchronize()
    assert ctx().device_errors() == 0
    Ss = db.per_problem(plan.S)
    rng = np.random.default_rng(0)
    for b in rng.choice(db.B, size=12, replace=False):
        e, n_ex = _sampled(probs[b], Ss[b].astype(np.float64), M, C, 0, 16, rng)
        assert e.max() <= 1e-4, (b, e.max())
    w, stats = core.weights(ctx(), db, plan.S, W.LAMBDA)
    Vp = core.update(ctx(), db, M, C, 0, w)
    torch.cuda.synchronize()
    assert np.abs(plan.V_plus.cpu().numpy() - Vp.cpu().numpy()).max() <= 2e-5
    assert np.all(np.isfinite(plan.stats.cpu().numpy()))


def test_full_size_config4_sampled():
    """K=65536, T=100 with 64 obstacles: sampled costs of the plain rollout and of the
    plan vs the oracle; plan V+ vs the plain path."""
    p = prep([W.config4()], F32)[0]
    M, C = params(F32)
    db = core.DeviceBatch([p], dtype=F32)
    say("config4 full: K=65536 T=100 obstacles=64")
    S, w, stats, Vp = _plain(db, M, C, 0, W.LAMBDA)
    plan = core.Plan(ctx(), db, M, C, 0, W.LAMBDA, use_graph=True)
    plan.launch()
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    e, n_ex = _sampled(p, S.cpu().numpy().astype(np.float64), M, C, 0, 48, rng)
    assert e.max() <= 1e-4
    assert rel_err(plan.S.cpu().numpy(), S.cpu().numpy().astype(np.float64)).max() <= 1e-6
    assert np.abs(plan.V_plus.cpu().numpy() - Vp.cpu().numpy()).max() <= 2e-5
    assert ctx().device_errors() == 0


@pytest.mark.parametrize("lam", [1.0, 30.0, 1e4])
def test_update_sparse_and_dense_paths(lam):
    """The update takes its sparse path when few weights are non-zero (lambda = 1) and its
    dense path when all are (large lambda); both agree with the oracle given the weights."""
    probs = prep(ragged_problems(), F32)
    M, C = params(F32)
    db = core.DeviceBatch(probs, dtype=F32)
    say(f"update paths lambda={lam}")
    S, w, stats, Vp = _plain(db, M, C, 3, lam)
    plan = core.Plan(ctx(), db, M, C, 3, lam, use_graph=False)
    plan.launch()
    torch.cuda.synchronize()
    ws = db.per_problem(w)
    Vps = db.controls(Vp)
    for b, p in enumerate(probs):
        r = oracle_iteration(p, M, C, 3, lam)
        err = float(np.abs(Vps[b] - oracle.update(p.V, ws[b].astype(np.float64), r["eps"])).max())
        assert err <= 1e-5, (b, err)
    err = float(np.abs(plan.V_plus.cpu().numpy() - Vp.cpu().numpy()).max())
    assert err <= 2e-5, err


def test_autotune_picks_a_timed_candidate_and_caches(tmp_path):
    """The autotuner times the candidates it is given, returns the fastest, stores it
    under the batch's shape key and returns the stored entry on the next call; a plan
    with the tuned geometry computes the same costs as another one-sample-per-lane plan."""
    from paper_2302_11719_amd import autotune

    probs = prep(ragged_problems(), F32)
    M, C = params(F32)
    db = core.DeviceBatch(probs, dtype=F32)
    cache = str(tmp_path / "tune.json")
    cands = [dict(pipeline=-1, block=64, tile=128, grid=0), dict(pipeline=-1, block=256, tile=256, grid=0),
             dict(pipeline=-1, block=128, tile=128, grid=256)]
    say("autotune 3 candidates")
    r = autotune.tune(ctx(), db, M, C, 3, W.LAMBDA, cands=cands, reps=3, warmup=1, cache=cache)
    assert not r.cached and len(r.table) == 3
    assert r.best in [{k: c[k] for k in ("pipeline", "block", "tile", "grid")} for c in cands]
    assert r.best_ms == min(row["kernel_ms"] for row in r.table) > 0.0
    r2 = autotune.tune(ctx(), db, M, C, 3, W.LAMBDA, cands=cands, cache=cache)
    assert r2.cached and r2.best == r.best and r2.key == r.key
    tp = autotune.tuned_plan(ctx(), db, M, C, 3, W.LAMBDA, cache=cache, use_graph=False)
    # one sample per lane in every candidate: per-sample costs are bit-identical across geometries
    ref = core.Plan(ctx(), db, M, C, 3, W.LAMBDA, use_graph=False, pipeline=-1, block=256, tile=256)
    tp.launch()
    ref.launch()
    torch.cuda.synchronize()
    assert torch.equal(tp.S, ref.S)
    assert ctx().device_errors() == 0


def test_obstacles_moved_between_launches():
    """FP32 rollouts read the obstacles through padded slots written at every launch:
    obstacles moved in place between two launches are seen by the plain rollout and by
    the plan (both against the oracle with the moved obstacles)."""
    probs = prep(ragged_problems(), F32)
    M, C = params(F32)
    db = core.DeviceBatch(probs, dtype=F32)
    plan = core.Plan(ctx(), db, M, C, 5, W.LAMBDA, use_graph=True, pipeline=-1)
    b_obs = [b for b, p in enumerate(probs) if len(p.track.obs)]
    assert b_obs
    for move in range(2):
        say(f"moved obstacles, launch {move}")
        S = core.rollout(ctx(), db, M, C, 5)
        plan.launch()
        torch.cuda.synchronize()
        assert ctx().device_errors() == 0
        Ss, Sp = db.per_problem(S), db.per_problem(plan.S)
        for b in b_obs:
            r = oracle_iteration(probs[b], M, C, 5, W.LAMBDA)
            ok = band_mask(r["margin"], BAND, f'moved obstacles, problem {b}', Ss[b], r["S"])
            assert ok.sum() > 0
            assert rel_err(Ss[b], r["S"])[ok].max() <= 1e-4, (move, b)
            assert rel_err(Sp[b], r["S"])[ok].max() <= 1e-4, (move, b)
            band_mask(r["margin"], BAND, f'moved obstacles, plan, problem {b}', Sp[b], r["S"])
        if move == 0:
            # move every obstacle of those problems onto the start point's neighbourhood
            # (changes the costs), in place on the device and in the oracle's copy
            S_before = Ss
            for b in b_obs:
                o = probs[b].track.obs.copy()
                o[:, 0] = probs[b].x0[0] + 0.5 + 0.1 * np.arange(len(o))
                o[:, 1] = probs[b].x0[1] - 0.2
                probs[b].track.obs = o.astype(np.float32).astype(np.float64)
            new = np.concatenate([p.track.obs.reshape(-1, 4) for p in probs if len(p.track.obs)]).ravel()
            db.obs.copy_(torch.as_tensor(new, dtype=F32, device="cuda"))
    assert any(np.abs(Ss[b] - S_before[b]).max() > 0 for b in b_obs)
    plan.close()


def test_static_and_queued_grids_agree():
    """A grid as large as the tile list never touches the tile queue; a smaller grid pops
    it and re-arms it on the way out.  Both take the same tiles and combine them in tile
    order, so over a closed loop (shield, plant step and warm start in the launch) the
    two plans stay bit-identical, launch after launch."""
    probs = prep(ragged_problems(), F32)
    M, C = params(F32)
    dist = torch.as_tensor(W.disturbances(3, 8 * len(probs)).reshape(-1), dtype=F32, device="cuda")
    rep = dict(n_steps=3, step=0.05, objective=W.OBJ_SHIELD)
    dbs = [core.DeviceBatch(probs, dtype=F32) for _ in range(2)]
    probe = core.Plan(ctx(), dbs[0], M, C, 4, W.LAMBDA, block=256, tile=256, use_graph=False)
    n_tiles = probe.info()["n_tiles"]
    assert n_tiles > 2
    plans = [core.Plan(ctx(), dbs[i], M, C, 4, W.LAMBDA, block=256, tile=256, grid=g, repair=rep, execute=True,
                       dist=dist.view(8, -1), use_graph=False) for i, g in enumerate((n_tiles, 2))]
    assert [p.info()["grid"] for p in plans] == [n_tiles, 2]
    for step in range(4):
        say(f"static vs queued grid, launch {step}")
        for pl in plans:
            pl.launch()
        torch.cuda.synchronize()
        for name in ("x0", "V", "iter"):
            assert torch.equal(getattr(dbs[0], name), getattr(dbs[1], name)), (step, name)
        for name in ("S", "V_plus", "stats", "V_safe"):
            assert torch.equal(getattr(plans[0], name), getattr(plans[1], name)), (step, name)
    assert ctx().device_errors() == 0


@pytest.mark.parametrize("pipeline", [1, -1])
def test_one_problem_plan_matches_its_slot_in_a_batch(pipeline):
    """A one-problem plan takes the problem's dimensions from the offsets read at plan
    creation instead of reading the tile list and the offsets in every workgroup.  Over a
    closed loop (shield, plant step, warm start) it stays bit-identical to the same problem
    as the first of two in a plan of the same mode (same noise stream: problem index 0)."""
    p = prep([W.config1(K=1000, T=29, seed=2)], F32)[0]
    q = prep([W.config1(K=300, T=41, seed=5)], F32)[0]
    M, C = params(F32)
    rep = dict(n_steps=4, step=0.05, objective=W.OBJ_SHIELD)
    n_dist = 6
    d2 = torch.as_tensor(W.disturbances(7, 2 * n_dist).reshape(n_dist, 2, 2), dtype=F32, device="cuda")
    d1 = d2[:, :1, :].contiguous()
    db1 = core.DeviceBatch([p], dtype=F32)
    db2 = core.DeviceBatch([p, q], dtype=F32)
    kw = dict(repair=rep, execute=True, use_graph=False, pipeline=pipeline, block=0 if pipeline == 1 else 256)
    pl1 = core.Plan(ctx(), db1, M, C, 9, W.LAMBDA, dist=d1, **kw)
    pl2 = core.Plan(ctx(), db2, M, C, 9, W.LAMBDA, dist=d2, **kw)
    for step in range(4):
        say(f"one-problem plan vs batch slot pipeline={pipeline}, launch {step}")
        pl1.launch()
        pl2.launch()
        torch.cuda.synchronize()
        assert np.array_equal(db1.per_problem(pl1.S)[0], db2.per_problem(pl2.S)[0]), step
        for name in ("V_plus", "V_safe"):
            assert np.array_equal(db1.controls(getattr(pl1, name))[0], db2.controls(getattr(pl2, name))[0]), (step, name)
        assert torch.equal(pl1.stats.view(-1, 4)[0], pl2.stats.view(-1, 4)[0]), step
        assert torch.equal(db1.x0.view(-1, 6)[0], db2.x0.view(-1, 6)[0]), step
        assert np.array_equal(db1.controls(db1.V)[0], db2.controls(db2.V)[0]), step
        assert int(db1.iter[0]) == int(db2.iter[0]), step
    assert ctx().device_errors() == 0
