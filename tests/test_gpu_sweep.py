"""GPU runs of the closed-loop collision sweep: determinism, the shield with no
iterations equals the DCBF-cost controller, rates in range."""
import pytest

from paper_2302_11719_amd import sweep
from paper_2302_11719_amd import workloads as W

from gpu_helpers import band_mask, ctx, say

pytestmark = pytest.mark.gpu


def test_sweep_cells_deterministic_and_consistent():
    say("sweep: K=256 T=20, 8 runs x 15 steps, three controllers")
    a = sweep.run_cell(ctx(), 256, 20, "mppi", runs=8, steps=15, seed=3)
    b = sweep.run_cell(ctx(), 256, 20, "mppi", runs=8, steps=15, seed=3)
    assert a.collision_rate == b.collision_rate and a.collisions_per_run == b.collisions_per_run
    d = sweep.run_cell(ctx(), 256, 20, "mppi_dcbf", runs=8, steps=15, seed=3)
    s0 = sweep.run_cell(ctx(), 256, 20, "shield", runs=8, steps=15, seed=3,
                        repair=dict(n_steps=0, step=0.05, objective=W.OBJ_SHIELD))
    assert s0.collision_rate == d.collision_rate and s0.collisions_per_run == d.collisions_per_run
    s = sweep.run_cell(ctx(), 256, 20, "shield", runs=8, steps=15, seed=3)
    for c in (a, d, s):
        assert 0.0 <= c.collision_rate <= 1.0 and c.ms_per_step > 0.0
    assert ctx().device_errors() == 0


@pytest.mark.parametrize("controller", ["mppi", "mppi_dcbf", "shield"])
def test_sweep_runs_replayed_against_the_oracle(controller):
    """Two runs of one cell per controller (MPPI without the barrier penalty, MPPI with
    it, Shield-MPPI) stepped through the sweep's own plan, each step checked against the
    oracle from the device's state and controls (teacher forcing): sampled costs, V+
    given the device costs, the shield's output, and the disturbed plant step."""
    import numpy as np
    import torch

    import oracle
    from gpu_helpers import rel_err

    K, T, runs, steps = 256, 10, 2, 16
    cs = sweep.setup_cell(ctx(), K, T, controller, runs, steps, seed=5, v_goal=8.0)
    M, C, db = cs.model, cs.cost, cs.db
    fired = 0
    for k in range(steps):
        x_b = db.x0.cpu().numpy().astype(np.float64).reshape(runs, 6)
        V_b = [v.astype(np.float64) for v in db.controls(db.V)]
        it_b = db.iter.cpu().numpy().copy()
        say(f"sweep replay {controller} step {k}")
        cs.plan.launch()
        torch.cuda.synchronize()
        Ss = db.per_problem(cs.plan.S)
        Vp = db.controls(cs.plan.V_plus)
        Vs = db.controls(cs.plan.V_safe) if cs.repair else Vp
        x_a = db.x0.cpu().numpy().astype(np.float64).reshape(runs, 6)
        for r, p in enumerate(cs.probs):
            S_ref, eps, margin = oracle.rollout(M, C, p.track, x_b[r], V_b[r], K, cs.seed, r, int(it_b[r]))
            ok = band_mask(margin, 1e-3, f'step {k} run {r}', Ss[r], S_ref)
            assert rel_err(Ss[r], S_ref)[ok].max() <= 1e-4, (k, r)
            w_ref, _ = oracle.weights(Ss[r].astype(np.float64), cs.lam)
            assert np.abs(Vp[r] - oracle.update(V_b[r], w_ref, eps)).max() <= 1e-5, (k, r)
            if cs.repair:
                Vs_ref = oracle.repair(M, C, p.track, x_b[r], Vp[r].astype(np.float64), cs.repair["n_steps"],
                                       cs.repair["step"], cs.repair["objective"])
                assert np.abs(Vs[r] - Vs_ref).max() <= 1e-3 * max(1.0, np.linalg.norm(Vp[r])), (k, r)
                fired += int(not np.array_equal(Vs[r], Vp[r]))
            x_ref = oracle.execute(M, x_b[r], Vs[r][0].astype(np.float64), cs.dist[int(it_b[r]), r])
            assert np.abs(x_a[r] - x_ref).max() <= 1e-5, (k, r)
    say(f"  shield changed V+ in {fired} of {runs * steps} run-steps")
    if controller == "shield":
        assert fired >= 1  # the replay covers steps in which the shield acted
    cs.plan.close()
    assert ctx().device_errors() == 0
